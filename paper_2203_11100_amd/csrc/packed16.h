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
//   prof(jj, p)  fills p[0..R-1] with the packed scores of column jj
//   hdiag        H of the row above the strip at the column before the chunk;
//                leaves as that of the chunk's last column
//   up_h, up_f   H and F of the row above the strip, per column
//   emit(jj, h, f)  takes H and F of the strip's bottom row at column jj as
//                soon as the column is done
template <int R, class Prof, class Emit>
__device__ __forceinline__ void sweep_chunk(uint32_t (&H)[R], uint32_t (&E)[R], uint32_t& hdiag,
                                            const uint32_t (&up_h)[4], const uint32_t (&up_f)[4],
                                            uint32_t& best, uint32_t go, uint32_t ge, Prof prof,
                                            Emit emit) {
  static_assert(R % 2 == 0, "rows are taken in pairs for the maximum");
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    uint32_t p[R];
    prof(jj, p);
    uint32_t hd = hdiag;
    hdiag = up_h[jj];
    uint32_t F = up_f[jj];
    uint32_t hprev = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t h = cell_from_diag(hadd(hd, p[k]), E[k], F, go, ge);
      hd = H[k];
      H[k] = h;
      if (k & 1) best = hmax3(best, hprev, h);
      else hprev = h;
    }
    emit(jj, H[R - 1], F);
  }
}

// sweep_chunk with the profile reads issued one column ahead: while row pair
// k2 of column jj is computed, row pair k2 of column jj + 1 is read, so the
// reads' latency hides behind a column of arithmetic (the chunk's first
// column is read at its start).  The registers held stay those of one
// column: a row pair's old values die as its new ones are read.  (Reading
// the next chunk's first column during the last column as well keeps those
// registers live across the chunk boundary and spills.)
//   prof_pair(jj, k2, a, b)  reads row pair k2 of column jj: with kSplit,
//                a = the low table's two (S, 1) dwords and b = the high
//                table's two (1, S) dwords, one fused multiply-add per cell
//                forming H_diag + S (see hfma); without, a = the two rows'
//                packed scores, added to H_diag (b unused)
//   emit(jj, h, f)  takes H and F of the strip's bottom row at column jj as
//                soon as the column is done (stored at once, the registers
//                of the four columns' results are not held to the chunk's end)
template <int R, bool kSplit, class ProfPair, class Emit>
__device__ __forceinline__ void sweep_chunk_ahead(uint32_t (&H)[R], uint32_t (&E)[R],
                                                  uint32_t& hdiag, const uint32_t (&up_h)[4],
                                                  const uint32_t (&up_f)[4], uint32_t& best,
                                                  uint32_t go, uint32_t ge, ProfPair prof_pair,
                                                  Emit emit) {
  static_assert(R % 2 == 0, "rows are taken in pairs");
  // VALU and SALU may cross the scheduling barriers; LDS reads may not
  constexpr int kMayCross = 0x0002 | 0x0004;
  uint2 a[R / 2], b[R / 2];
#pragma unroll
  for (int k2 = 0; k2 < R / 2; ++k2) prof_pair(0, k2, a[k2], b[k2]);
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    uint32_t hd = hdiag;
    hdiag = up_h[jj];
    uint32_t F = up_f[jj];
#pragma unroll
    for (int k2 = 0; k2 < R / 2; ++k2) {
      // an empty asm taking the F that enters the row pair keeps the first
      // use of its scores (read a column earlier) where the F chain reaches it
      if (kSplit) asm volatile("" : "+v"(a[k2]), "+v"(b[k2]) : "v"(F));
      else asm volatile("" : "+v"(a[k2]) : "v"(F));
      const uint2 ca = a[k2], cb = b[k2];
      if (jj < 3) {
        prof_pair(jj + 1, k2, a[k2], b[k2]);
        __builtin_amdgcn_sched_barrier(kMayCross);
      }
      const uint32_t d0 = kSplit ? hfma(ca.x, cb.x, hd) : hadd(hd, ca.x);
      const uint32_t h0 = cell_from_diag(d0, E[2 * k2], F, go, ge);
      hd = H[2 * k2];
      H[2 * k2] = h0;
      const uint32_t d1 = kSplit ? hfma(ca.y, cb.y, hd) : hadd(hd, ca.y);
      const uint32_t h1 = cell_from_diag(d1, E[2 * k2 + 1], F, go, ge);
      hd = H[2 * k2 + 1];
      H[2 * k2 + 1] = h1;
      best = hmax3(best, h0, h1);
    }
    emit(jj, H[R - 1], F);
  }
}

}  // namespace swdb
