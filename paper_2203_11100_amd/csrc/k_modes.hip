// Global and semi-global alignment scores of one query against every
// database sequence (other alignment operations beside the local search; the
// paper lists them for SW#, section 2.3, and as future work, section 5).
//
// Both are Gotoh's recurrence without the 0 in H's maximum:
//     E(i,j) = max(E(i,j-1) - ge, H(i,j-1) - go)
//     F(i,j) = max(F(i-1,j) - ge, H(i-1,j) - go)
//     H(i,j) = max(H(i-1,j-1) + S(a_i, b_j), E(i,j), F(i,j))
// with H(i,0) = -w(i) (the query's leading residues form one gap), H(0,j) =
// -w(j) in global mode and 0 in semi-global mode (the database sequence's
// leading residues are free there), E(i,0) = F(0,j) = -infinity, w(k) =
// go + (k-1) ge and w(0) = 0.  The score is H(m, n) (global) or
// max_{1<=j<=n} H(m, j) (semi-global: its trailing residues are free too),
// and H(m, 0) = -w(m) when the sequence is empty.  Scores are exact 32-bit
// integers; the host rejects gap penalties and lengths whose scores could
// leave +-2^28 (kModeRange), so -2^29 stands in for -infinity without
// overflow.
//
// k_mode_inter: inter-task form for the short bins.  Lane l of a wave owns
// one sequence (slot 64*half + l of a bin of the interleaved store) and
// sweeps the query in strips of R rows held in registers, column by column
// over the bin's padded length; the strip's bottom row (H and F per column)
// goes through a per-bin boundary buffer [len][128 slots] of int2 to the
// next strip, read and rewritten in place (each lane reads a column before
// it writes it).  Each wave runs alone (no workgroup barriers): four waves of
// a workgroup take four half bins.  The strip's profile is an int32
// [26 codes][R rows] table staged in the wave's own LDS buffer; the residue
// bytes hold 8 x code, so a byte times R/2 is the byte offset of the code's
// row.  Per cell: one add, one three-input max, three subtractions and two
// maxima.  Columns past a sequence's end see the pad code and rows past the
// query's end the pad score; neither reaches a real cell (they lie below or
// to the right of every real cell), and the score is read at the query's
// last row and the sequence's own columns only.
#include "internal.h"

namespace swdb {
namespace {

constexpr int kNegInf = -(1 << 29);

__device__ __forceinline__ int gapw(int k, int go, int ge) { return k == 0 ? 0 : go + (k - 1) * ge; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imax3(int a, int b, int c) { return imax(imax(a, b), c); }

// int32 profile [strip][26][R] (codes 0..23, the pad code, a spare) and the
// intra-task int8 profile [25][m_pad2] of the long-sequence kernel.
__global__ void k_mode_profile(const uint8_t* __restrict__ q, int m, Matrix mat, int R,
                               int n_strips, int32_t* __restrict__ prof, int8_t* __restrict__ prof2,
                               int m_pad2) {
  const int64_t n1 = (int64_t)n_strips * kProfRowDwords * R;
  const int64_t n2 = (int64_t)kIntraCodes * m_pad2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n1 + n2;
       idx += stride) {
    int i, c;
    if (idx < n1) {
      const int r = (int)(idx % R);
      const int64_t sc = idx / R;
      c = (int)(sc % kProfRowDwords);
      i = (int)(sc / kProfRowDwords) * R + r;
    } else {
      const int64_t j = idx - n1;
      c = (int)(j / m_pad2);
      i = (int)(j % m_pad2);
    }
    int v = kPadScore;
    if (i < m && c < SW_ALPHA) {
      const int qc = q[i];
      if (qc < SW_ALPHA) v = mat.v[qc * SW_ALPHA + c];
    }
    if (idx < n1) prof[idx] = v;
    else prof2[idx - n1] = (int8_t)v;
  }
}

// Scores of every sequence against an empty query: -w(n) (global), 0
// (semi-global).
__global__ void k_mode_empty_query(const int64_t* __restrict__ offs, int64_t n_seqs, int mode,
                                   int go, int ge, int32_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_seqs; s += stride)
    out[s] = mode == SW_MODE_GLOBAL ? -gapw((int)(offs[s + 1] - offs[s]), go, ge) : 0;
}

template <int R, int MODE>
__global__ __launch_bounds__(256) void k_mode_inter(ModeArgs a) {
  constexpr int RS = R + 4;   // LDS stride of a code's row, dwords
  __shared__ __align__(16) int32_t lprof_all[4][kProfRowDwords * RS];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int hb = blockIdx.x * 4 + w;
  if (hb >= a.n_halfbins) return;     // the whole wave
  int32_t* lprof = &lprof_all[w][0];
  const BinDesc bd = a.bins[hb >> 1];
  const int slot = (hb & 1) * 64 + lane;
  const int sid = a.slot_seq[bd.slot0 + slot];
  const int n = sid >= 0 ? (int)(a.offs[sid + 1] - a.offs[sid]) : 0;
  const int L = (int)bd.len;
  const uint32_t* __restrict__ res = a.res + bd.res_off + slot;   // + (j / 4) * 128
  int2* __restrict__ rb = a.rb + 4 * bd.res_off + slot;            // + j * 128
  const int go = a.go, ge = a.ge, m = a.m;
  const int S = a.n_strips;
  const int kstar = (m - 1) % R;    // the query's last row within the last strip
  int score = kNegInf;

  for (int s = 0; s < S; ++s) {
    {  // stage the strip's profile (read back only by this wave)
      const int32_t* __restrict__ src = a.prof + (size_t)s * kProfRowDwords * R;
      constexpr int N = kProfRowDwords * R, IT = (N + 63) / 64;
      int32_t v[IT];   // every load in flight before the first write
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int x = it * 64 + lane;
        v[it] = x < N ? src[x] : 0;
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int x = it * 64 + lane;
        if (x < N) lprof[(x / R) * RS + x % R] = v[it];
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    const bool first = s == 0, last = s == S - 1;
    const int row0 = s * R;           // rows row0 + 1 .. row0 + R (1-based)
    int H[R], E[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      H[k] = -gapw(row0 + k + 1, go, ge);     // H(i, 0)
      E[k] = H[k] - go;                       // E(i, 1)
    }
    int hdiag = -gapw(row0, go, ge);          // H(row0, 0)
    // the row above each chunk of 4 columns, loaded one chunk ahead.  The
    // loads are issued on every path (the first strip discards them for the
    // top border) so that no branch around them makes a later wait drain
    // every outstanding store.
    auto load_up = [&](int j0, int2 (&u)[4], uint32_t& rw) {
      rw = res[(size_t)(j0 >> 2) * 128];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int2 v = rb[(size_t)(j0 + q) * 128];
        // the top border H(0, j) and the F it feeds into row 1:
        // max(F(0, j) - ge, H(0, j) - go) = H(0, j) - go
        const int top = MODE == SW_MODE_GLOBAL ? -gapw(j0 + q + 1, go, ge) : 0;
        u[q].x = first ? top : v.x;
        u[q].y = first ? top - go : v.y;
      }
    };
    int2 up_n[4];
    uint32_t rw_n;
    load_up(0, up_n, rw_n);
    // the profile column of the next database column is read from LDS one
    // column ahead, so that its latency hides behind a column of cells
    int PA[R], PB[R];
    auto load_prof = [&](uint32_t byte, int (&P)[R]) {
      const int32_t* pp = lprof + ((byte >> 3) & 31u) * RS;
#pragma unroll
      for (int k = 0; k < R; ++k) P[k] = pp[k];
    };
    load_prof(rw_n & 0xffu, PA);
    for (int j0 = 0; j0 < L; j0 += 4) {
      int2 up[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) up[q] = up_n[q];
      const uint32_t rw = rw_n;
      load_up(j0 + 4 < L ? j0 + 4 : j0, up_n, rw_n);   // past the end: this chunk again
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + q;
        int (&P)[R] = (q & 1) ? PB : PA;
        // column j + 1's code: the next byte of this chunk's word, else the
        // first byte of the next chunk's (this chunk's again past the last)
        load_prof(q < 3 ? (rw >> (8 * (q + 1))) & 0xffu : rw_n & 0xffu, (q & 1) ? PA : PB);
        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the cells
        int hd = hdiag;
        hdiag = up[q].x;
        int F = up[q].y;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const int h = imax3(hd + P[k], E[k], F);
          hd = H[k];
          H[k] = h;
          const int t = h - go;
          E[k] = imax(E[k] - ge, t);
          F = imax(F - ge, t);
        }
        // the strip's bottom row for the next one (written in the last strip
        // too, where nothing reads it: a store on every path)
        rb[(size_t)j * 128] = make_int2(H[R - 1], F);
        if (last) {
          int v = H[0];
#pragma unroll
          for (int k = 1; k < R; ++k) v = k == kstar ? H[k] : v;
          if (MODE == SW_MODE_GLOBAL) score = j == n - 1 ? v : score;
          else score = j < n ? imax(score, v) : score;
        }
      }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  if (sid >= 0) a.out[sid] = n == 0 ? -gapw(m, go, ge) : score;
}

template <int R, int MODE>
hipError_t launch_mode_rm(int grid, const ModeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_mode_inter<R, MODE>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mode_profile(const uint8_t* d_query, int m, const Matrix& mat, int R,
                               int n_strips, int32_t* prof, int8_t* prof2, int m_pad2,
                               hipStream_t s) {
  const int64_t total = (int64_t)n_strips * kProfRowDwords * R + (int64_t)kIntraCodes * m_pad2;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 2048));
  hipLaunchKernelGGL(k_mode_profile, dim3(grid), dim3(256), 0, s, d_query, m, mat, R, n_strips,
                     prof, prof2, m_pad2);
  return hipGetLastError();
}

hipError_t launch_mode_empty_query(const int64_t* offs, int64_t n_seqs, int mode, int go, int ge,
                                   int32_t* out, hipStream_t s) {
  if (n_seqs <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n_seqs + 255) / 256, 4096);
  hipLaunchKernelGGL(k_mode_empty_query, dim3(grid), dim3(256), 0, s, offs, n_seqs, mode, go, ge,
                     out);
  return hipGetLastError();
}

hipError_t launch_mode_inter(int R, int mode, const ModeArgs& a, hipStream_t s) {
  if (a.n_halfbins <= 0) return hipSuccess;
  const int grid = (a.n_halfbins + 3) / 4;
#define SWDB_CASE(r, md) \
  if (R == r && mode == md) return launch_mode_rm<r, md>(grid, a, s);
  SWDB_CASE(16, SW_MODE_GLOBAL) SWDB_CASE(32, SW_MODE_GLOBAL)
  SWDB_CASE(16, SW_MODE_SEMIGLOBAL) SWDB_CASE(32, SW_MODE_SEMIGLOBAL)
#undef SWDB_CASE
  return hipErrorInvalidValue;
}

}  // namespace swdb
