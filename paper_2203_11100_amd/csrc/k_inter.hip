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
// The query profile rows of the current strip are staged in LDS as two
// tables (internal.h, prof_strip_dwords): the low table holds (S(a_i, c), 1)
// and the high table (1, S(a_i, c)) as binary16, for 26 codes (24 residues,
// pad, spare), rows in pairs and code-major within a pair.  Per row pair a
// lane reads one 64-bit entry for its low sequence's residue x from the low
// table and one for its high sequence's residue y from the high table; the
// packed product (S(a_i, x), 1) * (1, S(a_i, y)) is (S(a_i, x), S(a_i, y)),
// so one packed fused multiply-add per cell forms H_diag + S for both
// sequences, with no byte permute.  All lanes read the same row pair, so the
// addresses fall in one 208-byte row pair of each table (two codes share a
// pair of 32-bit banks when they are 16 apart).  Each column's entries are
// read while the previous column is computed (sweep_chunk_ahead), so the
// LDS latency hides behind a column of arithmetic.  The next strip's rows
// are copied in during the current strip's last chunks, one or two dwords
// per lane per chunk, so the copy holds few registers.
#include "internal.h"
#include "packed16.h"

namespace swdb {
namespace {

template <int R, int W>
__global__ __launch_bounds__(64 * W) void k_inter_f16(InterArgs a) {
  constexpr int D = 2;   // superstep skew between consecutive waves
  constexpr int kSlot = prof_strip_dwords(R);
  constexpr int kHighBytes = R * kProfRowDwords * 4;   // the high table's offset
  constexpr int kStage = (kSlot + 63) / 64;            // dwords per lane per strip
  constexpr int kPer = (kStage + 15) / 16;             // staged per chunk
  constexpr int kStageChunks = (kStage + kPer - 1) / kPer;
  static_assert(kStageChunks <= SW_MIN_BIN_LEN / 4, "the staging needs kStageChunks chunks");
  __shared__ __attribute__((aligned(16))) uint32_t lprof[W][2][kSlot];
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
  uint4* __restrict__ rbb = a.rb + (bin.rb_off - a.rb_base);
  const uint32_t go = a.go2, ge = a.ge2;

  // inputs of the next chunk, fetched one superstep ahead.  The first strip
  // reads the boundary buffer too: every bin's buffer holds zeros between
  // searches (zeroed when allocated, and the last strip of every search
  // writes zeros in place of its bottom row), so every chunk issues the
  // same memory operations and the compiler can count them exactly.
  uint2 rr_n = make_uint2(0, 0);
  uint4 b0_n = make_uint4(0, 0, 0, 0), b1_n = make_uint4(0, 0, 0, 0);
  auto fetch = [&](int c) {
    rr_n = rbin[c * 64 + lane];
    const uint4* p = rbb + (size_t)(c * 64 + lane) * 2;
    b0_n = p[0];
    b1_n = p[1];
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
  if (w == 0 && my_rounds > 0) fetch(0);
  for (int T = 0; T < lead; ++T) {
    if (T == D * w - 1 && my_rounds > 0) fetch(0);
    __syncthreads();
  }
  // one 64-bit LDS read per row pair and sequence gives both rows' dwords,
  // (S, 1) from the low table for the low half's residue and (1, S) from the
  // high table for the high half's (two reads per ds_read2_b64 where they
  // pair); the residue bytes hold 8 x code, the byte offset of the code's
  // dword pair in a row pair
  auto read_pair = [&](const uint32_t* sl, uint2 res, int jj, int k2, uint2& A, uint2& B) {
    const uint2* plo = reinterpret_cast<const uint2*>(
        reinterpret_cast<const char*>(sl) + ((res.x >> (8 * jj)) & 0xffu));
    const uint2* phi = reinterpret_cast<const uint2*>(
        reinterpret_cast<const char*>(sl) + kHighBytes + ((res.y >> (8 * jj)) & 0xffu));
    A = plo[k2 * kProfRowDwords];
    B = phi[k2 * kProfRowDwords];
  };
  for (int q = 0; q < my_rounds; ++q) {
    const int s = q * Wu + w;
#pragma unroll
    for (int k = 0; k < R; ++k) { H[k] = 0; E[k] = 0; }
    uint32_t hdiag = 0;
    const uint32_t* slot = &lprof[w][q & 1][0];
    const bool more = q + 1 < my_rounds;
    // no scalar load may be pending when the chunk loop starts: scalar loads
    // return out of order, so one pending at the loop's entry would make the
    // compiler wait for all LDS reads at every chunk's start instead of only
    // for the first row pair's
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0), other counters untouched
    for (int c = 0; c < C; ++c) {
      const uint2 rr = rr_n;
      const uint32_t up_h[4] = {b0_n.x, b0_n.z, b1_n.x, b1_n.z};
      const uint32_t up_f[4] = {b0_n.y, b0_n.w, b1_n.y, b1_n.w};
      // the next chunk, or the first chunk of the next strip (after the last
      // strip a harmless reload of chunk 0)
      fetch(c + 1 < C ? c + 1 : 0);
      // next strip's profile, pieces kPer * x .. kPer * x + kPer - 1 of
      // kStage with x = c - (C - kStageChunks): the global loads now (always
      // issued, from this strip's own profile when there is nothing to
      // stage), the LDS stores after the compute
      const int x_st = c - (C - kStageChunks);
      const bool stage = more && x_st >= 0;
      const uint32_t* st_src = a.prof + (size_t)(stage ? s + Wu : s) * kSlot;
      uint32_t st[kPer];
#pragma unroll
      for (int y = 0; y < kPer; ++y)
        st[y] = st_src[min((kPer * max(x_st, 0) + y) * 64 + lane, kSlot - 1)];
      __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the compute
      // the strip's bottom row, (H, F) per column, stored as each column is
      // done (column jj at 8 jj bytes of the lane's 32-byte chunk entry)
      uint2* pbd = reinterpret_cast<uint2*>(rbb + (size_t)(c * 64 + lane) * 2);
      sweep_chunk_ahead<R, true>(H, E, hdiag, up_h, up_f, best, go, ge,
                                 [&](int jj, int k2, uint2& A, uint2& B) {
        read_pair(slot, rr, jj, k2, A, B);
      }, [&](int jj, uint32_t h, uint32_t f) { pbd[jj] = make_uint2(h, f); });
      // the last strip leaves zeros for the next search (the same lane's later
      // stores to the same addresses land last)
      if (s == S - 1) {
        uint4* pz = rbb + (size_t)(c * 64 + lane) * 2;
        pz[0] = make_uint4(0, 0, 0, 0);
        pz[1] = make_uint4(0, 0, 0, 0);
      }
      if (stage) {
#pragma unroll
        for (int y = 0; y < kPer; ++y) {
          const int o = (kPer * x_st + y) * 64 + lane;
          if (o < kSlot) lprof[w][(q + 1) & 1][o] = st[y];
        }
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
