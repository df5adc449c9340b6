// Batched inter-task Smith-Waterman/Gotoh kernel: many queries against the
// resident database in one persistent launch (paper section 2.2, database
// search; section 4.1 runs 20 queries against one database).
//
// Queries are sorted by length and paired; the two 16-bit halves of every
// register hold the two queries of a pair, scored against the same database
// sequence, so each lane owns one sequence and a wave 64.  The profile of a
// pair stores, for query row i and residue code c, the dword
// (S(a_i, c), S(b_i, c)), rows in pairs and code-major within a pair: one
// 64-bit LDS read per row pair returns both halves' scores for two rows with
// no packing op (all lanes read the same 208-byte row pair; codes 16 apart
// share a pair of banks).  The cell arithmetic, the R-row strips, the
// W-wave strip pipeline and the boundary-row handling are those of the
// single-query inter-task kernel (k_inter.hip).
//
// Work is a list of (pair, half bin) items, costliest first; a half bin is
// the 64 even or odd slots of a 128-sequence bin of the interleaved store.
// Each workgroup takes items from a device counter until the list is
// exhausted (every workgroup reaches the exit test after each item), and
// keeps one boundary-row buffer of its own for the item it is working on.
#include "internal.h"
#include "packed16.h"

namespace swdb {
namespace {

template <int R, int W>
__global__ __launch_bounds__(64 * W) void k_batch_f16(BatchArgs a) {
  constexpr int D = 2;   // superstep skew between consecutive waves
  constexpr int kSlot = R * kBatchRowDwords;
  constexpr int kStage = (kSlot + 63) / 64;
  static_assert(kStage <= SW_MIN_BIN_LEN / 4, "the staging needs kStage chunks per strip");
  __shared__ __attribute__((aligned(16))) uint32_t lprof[W][2][kSlot];
  __shared__ uint32_t lbest[W][64];
  __shared__ int litem;

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint4* __restrict__ rbb = a.rb + (size_t)blockIdx.x * a.rb_stride;
  const uint32_t go = a.go2, ge = a.ge2;

  for (;;) {
    if (threadIdx.x == 0) litem = atomicAdd(a.counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(litem);
    __syncthreads();
    if (it >= a.n_items) break;

    const int2 iv = a.items[it];
    const PairDesc pd = a.pairs[iv.x];
    const BinDesc bin = a.bins[iv.y >> 1];
    const int half = iv.y & 1;
    const int C = (int)(bin.len >> 2);
    const int S = pd.n_strips;
    // waves in use: the wrap from a round's last wave to the next round's
    // first needs C >= D * (Wu - 1) + 2 chunks (16 waves: shorter bins
    // leave the top waves idle; see k_inter.hip)
    const int Wu = __builtin_amdgcn_readfirstlane(min(W, C / D));
    const int q_last = (S - 1) / Wu, w_last = (S - 1) % Wu;
    const int T_total = q_last * C + D * w_last + C;
    const int my_rounds = (w < S && w < Wu) ? (S - 1 - w) / Wu + 1 : 0;
    const uint32_t* __restrict__ prof = a.prof + pd.prof_off;
    // lane's residues: dword res_off + c*128 + 2*lane + half
    const uint32_t* __restrict__ rlane = a.res + bin.res_off + 2 * lane + half;

    if (my_rounds > 0) {
      const uint32_t* src = prof + (size_t)w * kSlot;
#pragma unroll
      for (int x = 0; x < kStage; ++x)
        if (x * 64 + lane < kSlot) lprof[w][0][x * 64 + lane] = src[x * 64 + lane];
    }
    __syncthreads();

    uint32_t rr_n = 0;
    uint4 b_n = make_uint4(0, 0, 0, 0), b_n2 = make_uint4(0, 0, 0, 0);
    auto fetch = [&](int s, int c) {
      rr_n = rlane[(size_t)c * SW_BIN_SEQS];
      if (s > 0) {
        const uint4* p = rbb + (size_t)(c * 64 + lane) * 2;
        b_n = p[0];
        b_n2 = p[1];
      } else {
        b_n = make_uint4(0, 0, 0, 0);
        b_n2 = make_uint4(0, 0, 0, 0);
      }
    };

    uint32_t H[R], E[R];
    uint32_t best = 0;
    // every wave passes exactly T_total barriers (idle waves: all lead-in)
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
      // nothing may be pending when the chunk loop starts: the compiler
      // merges the loop's entry with its back edge, so a load pending on
      // entry would make every chunk wait for all memory operations, the
      // prefetch it has just issued included, before its first cell
      __builtin_amdgcn_s_waitcnt(0);   // vmcnt(0) expcnt(0) lgkmcnt(0)
      for (int c = 0; c < C; ++c) {
        const uint32_t rr = rr_n;
        const uint32_t up_h[4] = {b_n.x, b_n.z, b_n2.x, b_n2.z};
        const uint32_t up_f[4] = {b_n.y, b_n.w, b_n2.y, b_n2.w};
        if (c + 1 < C) fetch(s, c + 1);
        else if (more) fetch(s + Wu, 0);
        // next strip's profile, piece x = c - (C - kStage) of kStage, one
        // dword per lane: the global load now, the LDS store after the compute
        const int x_st = c - (C - kStage);
        const bool stage = more && x_st >= 0 && x_st * 64 + lane < kSlot;
        uint32_t st = 0;
        if (stage) st = prof[(size_t)(s + Wu) * kSlot + x_st * 64 + lane];
        // the strip's bottom row, (H, F) per column, stored as each column is
        // done (column jj at 8 jj bytes of the lane's 32-byte chunk entry);
        // the last strip's are stored too, unread (a first strip never reads
        // the workgroup's buffer), so the chunk has no branch
        uint2* pbd = reinterpret_cast<uint2*>(rbb + (size_t)(c * 64 + lane) * 2);
        // residue bytes hold 8 x code, the byte offset of the code's dword
        // pair in a row pair: one 64-bit LDS read gives two rows (reading a
        // column ahead, as the single-query kernel does, measured 2 % slower
        // here: one table, half the reads to hide)
        sweep_chunk<R>(H, E, hdiag, up_h, up_f, best, go, ge,
                       [&](int jj, uint32_t (&p)[R]) {
          const uint2* pc = reinterpret_cast<const uint2*>(
              reinterpret_cast<const char*>(slot) + ((rr >> (8 * jj)) & 0xffu));
#pragma unroll
          for (int k2 = 0; k2 < R / 2; ++k2) {
            const uint2 A = pc[k2 * kBatchRowDwords];
            p[2 * k2] = A.x;
            p[2 * k2 + 1] = A.y;
          }
        }, [&](int jj, uint32_t h, uint32_t f) { pbd[jj] = make_uint2(h, f); });
        if (stage) lprof[w][(q + 1) & 1][x_st * 64 + lane] = st;
        __syncthreads();
      }
    }
    for (int T = lead + my_rounds * C; T < T_total; ++T) __syncthreads();

    lbest[w][lane] = best;
    __syncthreads();
    if (w == 0) {
      uint32_t top = lbest[0][lane];
#pragma unroll
      for (int x = 1; x < W; ++x) top = hmax2(top, lbest[x][lane]);
      const int sid = a.slot_seq[bin.slot0 + 2 * lane + half];
      if (sid >= 0) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int qi = hh ? pd.qb : pd.qa;
          if (qi < 0) continue;
          const int score = half_score(top, hh, a.sat_limit);
          if (score < 0) {
            const int idx = atomicAdd(a.flag_count, 1);
            a.flag_list[idx] = make_int2(sid, qi);
          } else {
            a.out[(size_t)qi * a.n_seqs + sid] = score;
          }
        }
      }
    }
  }
}

template <int R, int W>
hipError_t launch_rw(int grid, const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_f16<R, W>), dim3(grid), dim3(64 * W), 0, s, a);
  return hipGetLastError();
}

template <int R, int W>
int occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_batch_f16<R, W>),
                                                   64 * W, 0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

}  // namespace

hipError_t launch_batch(int R, int W, int grid, const BatchArgs& a, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define SWDB_CASE(r, w) \
  if (R == r && W == w) return launch_rw<r, w>(grid, a, s);
  SWDB_CASE(16, 4) SWDB_CASE(16, 8) SWDB_CASE(16, 12) SWDB_CASE(32, 4) SWDB_CASE(32, 8)
  SWDB_CASE(12, 12) SWDB_CASE(14, 12) SWDB_CASE(18, 12) SWDB_CASE(20, 12) SWDB_CASE(12, 16) \
  SWDB_CASE(14, 16)
#undef SWDB_CASE
  return hipErrorInvalidValue;
}

int batch_workgroups_per_cu(int R, int W) {
#define SWDB_CASE(r, w) \
  if (R == r && W == w) return occupancy<r, w>();
  SWDB_CASE(16, 4) SWDB_CASE(16, 8) SWDB_CASE(16, 12) SWDB_CASE(32, 4) SWDB_CASE(32, 8)
  SWDB_CASE(12, 12) SWDB_CASE(14, 12) SWDB_CASE(18, 12) SWDB_CASE(20, 12) SWDB_CASE(12, 16) \
  SWDB_CASE(14, 16)
#undef SWDB_CASE
  return 1;
}

}  // namespace swdb
