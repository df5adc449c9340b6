// Packed half-precision cell arithmetic shared by the inter-task kernels.  A
// 32-bit register holds two independent cells (bits 0..15 and 16..31) as
// IEEE binary16 values.
//
// Exactness.  Every quantity of the recurrence is an integer, and binary16
// holds every integer of magnitude <= 2048 exactly, so sums, differences and
// maxima of such values are exact while they stay in that range.  Let the
// rescoring limit be L <= 2048 and the gap penalties o, e <= 2048 (larger
// ones are passed as 2048: in the exact regime H < 2048, so H - o and
// E - e are negative either way and meet a max with 0).  Suppose every
// cell that (i, j) depends on has H < L and was computed exactly.  Then
// E(i, j) and F(i, j) are maxima of 0 and differences of integers in
// [0, 2048], all exact and below L; and H_diag + S, exact or not, is at most
// the true H(i, j).  So if the true H(i, j) < L, the sum is below 2048 and
// exact, and H(i, j) is exact; if the true H(i, j) >= L, then H_diag + S >= L
// and its rounding (monotone, 2048 representable) is still >= L, so the
// computed maximum reaches L.  By induction: a sequence whose true score is
// below L is scored exactly, and one whose score is L or more ends with a
// computed maximum >= L and is rescored exactly in 32-bit integers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swdb {

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h16x2 as_h2(uint32_t a) { return __builtin_bit_cast(h16x2, a); }
__device__ __forceinline__ uint32_t as_u32(h16x2 a) { return __builtin_bit_cast(uint32_t, a); }

// per half: a + b, a - b (v_pk_add_f16)
__device__ __forceinline__ uint32_t hadd(uint32_t a, uint32_t b) { return as_u32(as_h2(a) + as_h2(b)); }
__device__ __forceinline__ uint32_t hsub(uint32_t a, uint32_t b) { return as_u32(as_h2(a) - as_h2(b)); }
// per half: a * b + c (v_pk_fma_f16).  With a = (S_x, 1) and b = (1, S_y)
// it is c + (S_x, S_y): the products by 1 are exact and the sum rounds
// once, exactly as the add would.
__device__ __forceinline__ uint32_t hfma(uint32_t a, uint32_t b, uint32_t c) {
  return as_u32(__builtin_elementwise_fma(as_h2(a), as_h2(b), as_h2(c)));
}
// per half: max(a, b) and max(a, b, c) (v_pk_maximum3_f16)
__device__ __forceinline__ uint32_t hmax2(uint32_t a, uint32_t b) {
  return as_u32(__builtin_elementwise_maximum(as_h2(a), as_h2(b)));
}
__device__ __forceinline__ uint32_t hmax3(uint32_t a, uint32_t b, uint32_t c) {
  return as_u32(__builtin_elementwise_maximum(__builtin_elementwise_maximum(as_h2(a), as_h2(b)),
                                              as_h2(c)));
}

// Score in one half of a register of maxima, as an integer, or -1 when it
// reaches `limit` (infinity included) and the sequence must be rescored.
__device__ __forceinline__ int half_score(uint32_t v, int half, int limit) {
  const float f = (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> (16 * half)));
  return f < (float)limit ? (int)f : -1;
}

// One cell of Gotoh's recurrence on both halves, with E and F kept as
// max(E, 0) and max(F, 0) (then H = max(H_diag + S, E, F) needs no 0):
//   h = max(d, E, F);  t = h - o;  E = max(E - e, t, 0);  F = max(F - e, t, 0)
// where d = H(i-1, j-1) + S(a_i, b_j).  Returns h.
__device__ __forceinline__ uint32_t cell_from_diag(uint32_t d, uint32_t& E, uint32_t& F,
                                                   uint32_t go, uint32_t ge) {
  const uint32_t h = hmax3(d, E, F);
  const uint32_t t = hsub(h, go);
  E = hmax3(hsub(E, ge), t, 0u);
  F = hmax3(hsub(F, ge), t, 0u);
  return h;
}

// The cell with packed scores p: hd enters as H(i-1, j-1) and leaves as
// H(i, j-1) (the next row's diagonal); H enters as H(i, j-1) and leaves as
// H(i, j).  Returns h.
__device__ __forceinline__ uint32_t cell(uint32_t& hd, uint32_t& H, uint32_t& E, uint32_t& F,
                                         uint32_t p, uint32_t go, uint32_t ge) {
  const uint32_t h = cell_from_diag(hadd(hd, p), E, F, go, ge);
  hd = H;
  H = h;
  return h;
}

// Scores one 4-column chunk of an R-row strip, column by column.  The
// running maximum takes two rows per 3-input max.  (Sweeping bands of two or
// four columns along anti-diagonals, which removes the wait states between
// dependent packed ops, measured 5 % and 7 % slower on gfx950.)
//   prof(jj, p, p2)  fills, for column jj, p[0..R-1] with the packed scores
//                (kSplit false), or p with the (S, 1) dwords of the low half's
//                residue and p2 with the (1, S) dwords of the high half's
//                (kSplit true: one fused multiply-add per cell forms
//                H_diag + S, see hfma)
//   hdiag        H of the row above the strip at the column before the chunk;
//                leaves as that of the chunk's last column
//   up_h, up_f   H and F of the row above the strip, per column
//   out_h, out_f H and F of the strip's bottom row, per column
template <int R, bool kSplit, class Prof>
__device__ __forceinline__ void sweep_chunk(uint32_t (&H)[R], uint32_t (&E)[R], uint32_t& hdiag,
                                            const uint32_t (&up_h)[4], const uint32_t (&up_f)[4],
                                            uint32_t (&out_h)[4], uint32_t (&out_f)[4],
                                            uint32_t& best, uint32_t go, uint32_t ge, Prof prof) {
  static_assert(R % 2 == 0, "rows are taken in pairs for the maximum");
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    uint32_t p[R], p2[R];
    prof(jj, p, p2);
    uint32_t hd = hdiag;
    hdiag = up_h[jj];
    uint32_t F = up_f[jj];
    uint32_t hprev = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t d = kSplit ? hfma(p[k], p2[k], hd) : hadd(hd, p[k]);
      const uint32_t h = cell_from_diag(d, E[k], F, go, ge);
      hd = H[k];
      H[k] = h;
      if (k & 1) best = hmax3(best, hprev, h);
      else hprev = h;
    }
    out_h[jj] = H[R - 1];
    out_f[jj] = F;
  }
}

}  // namespace swdb
