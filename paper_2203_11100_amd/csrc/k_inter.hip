// Inter-task Smith-Waterman/Gotoh kernel: every lane scores two database
// sequences against the query (paper section 2.2: inter-task parallelism,
// one independent alignment matrix per processing element, no communication
// between elements), in packed half-precision arithmetic.
//
// Cells follow Gotoh's recurrence over query rows i and database columns j:
//   E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o)
//   F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)
//   H(i,j) = max(0, H(i-1,j-1) + S(a_i,b_j), E(i,j), F(i,j)),  score = max H.
// E and F are kept as E' = max(E, 0), F' = max(F, 0): because H >= 0,
// max(E' - e, H - o, 0) = max(E - e, H - o, 0), so E' obeys the same update
// with a floor at 0, and H = max(H_diag + S, E', F') needs no separate 0.
// gfx950's 3-input packed maximum then gives a cell in 7 packed ops plus
// half of one for the running maximum.  The values are integers held in
// binary16, exact below the rescoring limit (packed16.h); sequences whose
// maximum reaches the limit are handed to the exact 32-bit kernel.
//
// Work decomposition.  A workgroup owns one bin of 128 length-sorted
// sequences (lane l holds the sequences of slots 2l and 2l+1 in the low and
// high 16-bit halves).  The query is cut into strips of R rows; the H and E
// state of a strip's R rows lives in registers while the strip sweeps every
// column of the bin.  The bottom row of a strip (H and the F flowing into
// the next row) is written to a per-bin boundary buffer and read back by the
// next strip.  The W waves of a workgroup take strips round robin and run
// as a pipeline: in superstep T, wave w works on columns 4c..4c+3 of its
// current strip, with c = T - 2w - q*C (q = its strip round, C = columns/4),
// and a workgroup barrier separates supersteps.  Strip s works on chunk c two
// supersteps after strip s-1, so it can prefetch the chunk's residues and
// boundary values one superstep ahead; the buffer can be overwritten in place
// because every strip reads a chunk before writing it.
// Splitting one bin's strips over W waves divides its latency by W, which
// keeps the longest bins from trailing the rest of the grid.
//
// The query profile rows of the current strip are staged in LDS as row pairs:
// dword (r, c) holds the scores of query rows 2r and 2r+1 against residue
// code c (26 codes: 24 residues, pad, spare).  All lanes read the same row
// pair at once, so the addresses fall in 26 consecutive dwords: no bank
// conflicts.  One read per row pair and half (lo/hi sequence) yields two
// rows; one byte permute per row packs the lo and hi sequences' scores.
#include "internal.h"
#include "packed16.h"

namespace swdb {
namespace {

template <int R, int W>
__global__ __launch_bounds__(64 * W) void k_inter_f16(InterArgs a) {
  constexpr int D = 2;   // superstep skew between consecutive waves
  constexpr int kSlot = R * kProfRowDwords;
  constexpr int kStage = (kSlot + 63) / 64;
  __shared__ uint32_t lprof[W][2][kSlot];
  __shared__ uint32_t lbest[W][64];

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const BinDesc bin = a.bins[a.bin_begin + blockIdx.x];
  const int C = (int)(bin.len >> 2);
  const int S = a.n_strips;
  // waves in use: the wrap from the last wave of a round to the first of the
  // next needs C >= D * (Wu - 1) + 2 chunks (see below), so a bin shorter
  // than that leaves the top waves idle (never with 12 waves: every bin has
  // at least SW_MIN_BIN_LEN / 4 = 24 chunks)
  const int Wu = __builtin_amdgcn_readfirstlane(min(W, C / D));
  const int q_last = (S - 1) / Wu, w_last = (S - 1) % Wu;
  const int T_total = q_last * C + D * w_last + C;
  const int my_rounds = (w < S && w < Wu) ? (S - 1 - w) / Wu + 1 : 0;

  if (my_rounds > 0) {
    const uint32_t* src = a.prof + (size_t)w * kSlot;
#pragma unroll
    for (int x = 0; x < kStage; ++x)
      if (x * 64 + lane < kSlot) lprof[w][0][x * 64 + lane] = src[x * 64 + lane];
  }
  __syncthreads();

  const uint2* __restrict__ rbin = a.res2 + (bin.res_off >> 1);
  uint4* __restrict__ rbb = a.rb + bin.rb_off;
  const uint32_t go = a.go2, ge = a.ge2;

  // inputs of the next chunk, fetched one superstep ahead
  uint2 rr_n = make_uint2(0, 0);
  uint4 b0_n = make_uint4(0, 0, 0, 0), b1_n = make_uint4(0, 0, 0, 0);
  auto fetch = [&](int s, int c) {
    rr_n = rbin[c * 64 + lane];
    if (s > 0) {
      const uint4* p = rbb + (size_t)(c * 64 + lane) * 2;
      b0_n = p[0];
      b1_n = p[1];
    } else {
      b0_n = make_uint4(0, 0, 0, 0);
      b1_n = make_uint4(0, 0, 0, 0);
    }
  };

  uint32_t H[R], E[R];
  uint32_t best = 0;

  // Wave w idles for D*w supersteps (prefetching in the last one), runs its
  // strips back to back, then idles until the last wave finishes; every wave
  // passes T_total barriers.  With the skew D = 2, the chunk a wave prefetches
  // in superstep T was written by the previous strip's wave in T-1 or
  // earlier; for the wrap from the last wave to the first that needs
  // C >= D * (Wu - 1) + 2, which is how Wu is chosen.
  // Every wave passes exactly T_total barriers: its lead-in (all of T_total
  // for an idle wave), my_rounds * C supersteps of work, then the tail.
  const int lead = min(D * w, T_total);
  if (w == 0 && my_rounds > 0) fetch(0, 0);
  for (int T = 0; T < lead; ++T) {
    if (T == D * w - 1 && my_rounds > 0) fetch(w, 0);
    __syncthreads();
  }
  for (int q = 0; q < my_rounds; ++q) {
    const int s = q * Wu + w;
#pragma unroll
    for (int k = 0; k < R; ++k) { H[k] = 0; E[k] = 0; }
    uint32_t hdiag = 0;
    const uint32_t* slot = &lprof[w][q & 1][0];
    const bool more = q + 1 < my_rounds;
    for (int c = 0; c < C; ++c) {
      const uint2 rr = rr_n;
      const uint32_t up_h[4] = {b0_n.x, b0_n.z, b1_n.x, b1_n.z};
      const uint32_t up_f[4] = {b0_n.y, b0_n.w, b1_n.y, b1_n.w};
      if (c + 1 < C) fetch(s, c + 1);
      else if (more) fetch(s + Wu, 0);
      // next strip's profile: global loads now, LDS stores after the compute
      const bool stage = more && c == C - 1;
      uint32_t st[kStage];
      if (stage) {
        const uint32_t* src = a.prof + (size_t)(s + Wu) * kSlot;
#pragma unroll
        for (int x = 0; x < kStage; ++x)
          if (x * 64 + lane < kSlot) st[x] = src[x * 64 + lane];
      }
      uint32_t out_h[4], out_f[4];
      // one 32-bit LDS read per row pair and sequence gives two rows'
      // scores; a byte permute per row packs the lo and hi sequences'.  The
      // residue bytes hold 4 x code, the code's byte offset in a row pair.
      sweep_chunk<R>(H, E, hdiag, up_h, up_f, out_h, out_f, best, go, ge,
                     [&](int jj, uint32_t (&p)[R]) {
        const uint32_t* plo = reinterpret_cast<const uint32_t*>(
            reinterpret_cast<const char*>(slot) + ((rr.x >> (8 * jj)) & 0xffu));
        const uint32_t* phi = reinterpret_cast<const uint32_t*>(
            reinterpret_cast<const char*>(slot) + ((rr.y >> (8 * jj)) & 0xffu));
#pragma unroll
        for (int k2 = 0; k2 < R / 2; ++k2) {
          const uint32_t A = plo[k2 * kProfPairDwords], B = phi[k2 * kProfPairDwords];
          // v_perm_b32: bytes {A0, A1, B0, B1} and {A2, A3, B2, B3}
          p[2 * k2] = __builtin_amdgcn_perm(B, A, 0x05040100u);
          p[2 * k2 + 1] = __builtin_amdgcn_perm(B, A, 0x07060302u);
        }
      });
      if (s < S - 1) {
        uint4* p = rbb + (size_t)(c * 64 + lane) * 2;
        p[0] = make_uint4(out_h[0], out_f[0], out_h[1], out_f[1]);
        p[1] = make_uint4(out_h[2], out_f[2], out_h[3], out_f[3]);
      }
      if (stage) {
#pragma unroll
        for (int x = 0; x < kStage; ++x)
          if (x * 64 + lane < kSlot) lprof[w][(q + 1) & 1][x * 64 + lane] = st[x];
      }
      __syncthreads();
    }
  }
  for (int T = lead + my_rounds * C; T < T_total; ++T) __syncthreads();

  lbest[w][lane] = best;
  __syncthreads();
  if (w != 0) return;
  uint32_t top = lbest[0][lane];
#pragma unroll
  for (int x = 1; x < W; ++x) top = hmax2(top, lbest[x][lane]);
  const int64_t slot0 = bin.slot0 + 2 * lane;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int sid = a.slot_seq[slot0 + half];
    if (sid < 0) continue;
    const int score = half_score(top, half, a.sat_limit);
    if (score < 0) {
      const int idx = atomicAdd(a.flag_count, 1);
      a.flag_list[idx] = make_int2(sid, 0);
    } else {
      a.out[sid] = score;
    }
  }
}

template <int R, int W>
hipError_t launch_rw(int n_bins, const InterArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_inter_f16<R, W>), dim3(n_bins), dim3(64 * W), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_inter(int R, int W, int n_bins, const InterArgs& a, hipStream_t s) {
  if (n_bins <= 0) return hipSuccess;
#define SWDB_CASE(r, w) \
  if (R == r && W == w) return launch_rw<r, w>(n_bins, a, s);
  SWDB_CASE(16, 1) SWDB_CASE(16, 2) SWDB_CASE(16, 4) SWDB_CASE(16, 8) SWDB_CASE(16, 12)
  SWDB_CASE(32, 1) SWDB_CASE(32, 2) SWDB_CASE(32, 4) SWDB_CASE(32, 8)
  SWDB_CASE(12, 12) SWDB_CASE(14, 12) SWDB_CASE(18, 12) SWDB_CASE(20, 12)
  SWDB_CASE(12, 16) SWDB_CASE(14, 16)
#undef SWDB_CASE
  return hipErrorInvalidValue;
}

}  // namespace swdb
