// Intra-task Smith-Waterman/Gotoh kernel for long database sequences and for
// exact 32-bit rescoring (paper section 2.2: intra-task parallelism, all
// processing elements work on one alignment matrix and neighbours exchange
// border elements; section 2.3: SW#db switches to it by sequence length).
//
// One workgroup of W2 waves scores one (query, database sequence) pair at a
// time, taking pairs from an item list (one query, or every query of a
// batch with per-query profile offsets).  The query is cut into passes of 64*R rows; lane l of a wave owns R
// consecutive rows of its pass and the wave sweeps the database sequence as
// an anti-diagonal wavefront: at step t lane l computes column j = t - l of
// its rows, so it receives the H and F values of row (top - 1) for column j
// from lane l-1, which computed them in the previous step.  That exchange is
// one cross-lane DPP move per value (wave_shr:1), with no LDS and no barrier
// inside the wave.  Lane 0 is fed the previous pass's bottom row (H and the F
// flowing into the next row) from a per-workgroup buffer, and the last lane's
// bottom row is collected (wave_shl:1) for the next pass.  Residue codes and
// the boundary row enter 64 columns at a time and move down the wave one
// lane per step.
//
// The W2 waves take passes round robin and run as a pipeline, like the
// strips of the inter-task kernel: a superstep is 64 steps, wave w runs
// superstep c of its pass q*W2 + w in workgroup superstep T = q*C2 + 3w + c,
// and workgroup barriers separate supersteps.  Pass p needs columns
// 64c..64c+63 of pass p-1's bottom row, which are complete once pass p-1 has
// finished its superstep c+1; the skew of 3 supersteps leaves one superstep
// for the prefetch of those columns.  Every pass has at least 3*W2 supersteps
// (short sequences are padded with pad columns), which covers the wrap from
// the last wave to the first.  The boundary buffer is overwritten in place:
// a pass reads each column before it writes it.
//
// Cells use the exact recurrence in 32-bit integers with E and F kept as
// max(E, 0), max(F, 0) (equivalent because H >= 0; see the inter-task
// kernel), so H = max(H_diag + S, E, F) is one three-input maximum.  Columns
// before a lane's first column and after the sequence's end see the pad code,
// whose profile score is <= 0, so they never raise the maximum.
//
// Column segments (packed kernel, short queries).  One long sequence's
// wavefront takes about n steps however few rows the query has, so for a
// short query the longest database sequence would set the search's time.
// The packed kernel can instead take items {pair, segment}: segment s
// covers columns [s*C, (s+1)*C) and is computed over a window starting
// `overlap` columns earlier, from a zero left border, as an independent
// local alignment of that window.  Every value computed there is a lower
// bound of the true one (fewer alignments are possible), and it is exact in
// the segment's own columns when every alignment of positive score ending
// there starts inside the window, which the host guarantees by the span
// bound at seg_overlap (runtime.hip).  The segments' maxima are combined per
// pair afterwards (k_long_combine), so segments of one sequence run on
// different workgroups at once.
//
// Each wave stages its pass's profile in LDS as int8 [code][row]: a lane
// reads its R rows for its own residue code, R contiguous bytes at
// code*64R + R*l, so the 64 reads of a wave cover consecutive bytes of one
// code row each and never conflict on banks.
#include "internal.h"
#include "packed16.h"

namespace swdb {
namespace {

constexpr int kWaveShr1 = 0x138;  // DPP wave_shr:1  (lane l <- lane l-1)
constexpr int kWaveShl1 = 0x130;  // DPP wave_shl:1  (lane l <- lane l+1)
constexpr int kSkew = 3;          // supersteps between consecutive passes

// lane l <- lane l-1; lane 0 keeps `first`
__device__ __forceinline__ int shr_in(int v, int first) {
  return __builtin_amdgcn_update_dpp(first, v, kWaveShr1, 0xf, 0xf, false);
}
// lane l <- lane l+1; lane 63 keeps `last`
__device__ __forceinline__ int shl_in(int v, int last) {
  return __builtin_amdgcn_update_dpp(last, v, kWaveShl1, 0xf, 0xf, false);
}

template <int R> struct ProfVec;
template <> struct ProfVec<2> { typedef uint16_t T; };
template <> struct ProfVec<4> { typedef uint32_t T; };
template <> struct ProfVec<8> { typedef uint2 T; };

// sign-extends the R int8 profile values of a lane
template <int R>
__device__ __forceinline__ void unpack_profile(const typename ProfVec<R>::T& v, int (&p)[R]);
template <>
__device__ __forceinline__ void unpack_profile<2>(const uint16_t& v, int (&p)[2]) {
  const int x = (int)v;
  p[0] = (x << 24) >> 24;
  p[1] = (x << 16) >> 24;
}
template <>
__device__ __forceinline__ void unpack_profile<4>(const uint32_t& v, int (&p)[4]) {
  const int x = (int)v;
#pragma unroll
  for (int k = 0; k < 4; ++k) p[k] = (x << (24 - 8 * k)) >> 24;
}
template <>
__device__ __forceinline__ void unpack_profile<8>(const uint2& v, int (&p)[8]) {
  const int x = (int)v.x, y = (int)v.y;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    p[k] = (x << (24 - 8 * k)) >> 24;
    p[k + 4] = (y << (24 - 8 * k)) >> 24;
  }
}

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// (score s, column c, row r) comes before (s2, c2, r2) as the end of a best
// alignment: a higher score, else the smaller column, else the smaller row
__device__ __forceinline__ bool end_before(int s, int c, int r, int s2, int c2, int r2) {
  return s > s2 || (s == s2 && (c < c2 || (c == c2 && r < r2)));
}

// kEnds: also find where the best local alignment ends - the cell (i, j)
// holding the maximum that comes first in database-then-query order
// (smallest column j, then smallest row i) - and write {sid, score, i, j}
// (0-based residue indices, -1 for a score of 0) to a.ends[item] instead of
// the score to a.out.  Within one pass a lane meets its cells in that order
// (columns advance with the step, rows with k inside a step), so a strict
// "greater" keeps the first; passes, lanes and waves are merged comparing
// (score, column, row).  Pad rows and columns never come first: with
// open > 0 a gap value stays below the maximum it came from, and with
// open = 0 a pad cell can only repeat a value some real cell earlier in
// (column, row) order already holds.
//
// kVarGlobal, kVarSemi: the global and semi-global scores of the same
// recurrence without the floor at 0 (the borders and score of each are
// stated where the inter-task form k_mode_inter is defined): the first pass
// is fed the top border row, every pass starts its rows at the left border,
// a lane keeps its rows at the border while its column is still negative
// (so the lane below reads the border as its diagonal), and the lane holding
// the query's last row reads the score from the sequence's own columns in
// the last pass.
//
// kVarTrace: kVarEnds plus one traceback code per cell (i, j), so that the
// host can walk an optimal alignment back from the end: bits 0-1 say where
// H(i, j) came from (0: it is 0, the alignment starts after this cell; 1:
// the diagonal H(i-1, j-1) + S; 3: F(i, j); 2: E(i, j); the first that
// equals H in the order 0, diagonal, F, E), bit 2 that E(i, j+1) comes from
// opening a gap after H(i, j) rather than extending E(i, j), bit 3 the same
// for F(i+1, j) (opening preferred on ties).  The clamped E and F give the
// same choices wherever the walk can be: it enters E or F only where they
// are positive, and a positive value never comes from a clamped 0.  Codes
// are bytes [column][row] (row = 0-based query position), one 8-, 4- or
// 2-byte store per lane and step for its R rows, written for the sequence's
// own columns only.
enum { kVarScore = 0, kVarEnds = 1, kVarGlobal = 2, kVarSemi = 3, kVarTrace = 4 };
constexpr int kNegInf = -(1 << 29);

__device__ __forceinline__ int gapw(int k, int go, int ge) { return k == 0 ? 0 : go + (k - 1) * ge; }

template <int R, int W2, int V>
__global__ __launch_bounds__(64 * W2) void k_intra_i32(IntraArgs a) {
  constexpr bool kTrace = V == kVarTrace;
  constexpr bool kEnds = V == kVarEnds || kTrace;
  constexpr bool kLocal = V == kVarScore || kEnds;
  constexpr int ROWS = 64 * R;   // query rows per pass
  __shared__ __align__(16) int8_t lprof_all[W2][kIntraCodes * ROWS];
  __shared__ int lbest[W2];
  __shared__ int lpos[kEnds ? 2 * W2 : 1];
  typedef typename ProfVec<R>::T PV;

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int8_t* lprof = &lprof_all[w][0];
  const int count = a.count_ptr ? *a.count_ptr : a.count;
  int2* __restrict__ rb = a.scratch + (size_t)blockIdx.x * a.scratch_stride;
  const int go = a.go, ge = a.ge;

  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    // kEnds with segments: item {hit, segment}; columns [c0, hi) of the hit
    // sequence as in the long-pair kernel's column segments
    const int2 sg = a.seg_items ? a.seg_items[it] : make_int2(it, 0);
    const int2 item = a.items[sg.x];
    const int sid = item.x;
    const QueryDesc qd = a.queries ? a.queries[item.y] : a.q0;
    const int P = qd.n_pass;
    const int q_last = (P - 1) / W2, w_last = (P - 1) % W2;
    const int my_rounds = (w < P) ? (P - 1 - w) / W2 + 1 : 0;
    const int8_t* __restrict__ qprof = a.prof2 + qd.prof2_off;
    const int64_t b0 = a.offs[sid];
    int n = (int)(a.offs[sid + 1] - b0);
    const uint8_t* __restrict__ bseq = a.res + b0;
    int c0 = 0;
    if (kEnds && a.seg_items) {
      const int lo = sg.y * a.seg_cols;
      const int hi = min(n, lo + a.seg_cols);
      c0 = max(0, lo - a.seg_overlap);
      n = max(hi - c0, 0);
      bseq += c0;
    }
    uint8_t* __restrict__ dir = kTrace ? a.dir + a.dir_off[it] : nullptr;
    // supersteps per pass: n + 63 steps, at least kSkew*W2 (see above)
    const int C2 = max((n + 63 + 63) >> 6, kSkew * W2);
    const int T_total = q_last * C2 + kSkew * w_last + C2;

    // feeder values of the next superstep, fetched one superstep ahead
    int fcode_n = SW_PAD_CODE, fh_n = 0, ff_n = 0;
    auto fetch = [&](int p, int c) {
      const int jf = c * 64 + lane;
      fcode_n = jf < n ? (int)bseq[jf] : SW_PAD_CODE;
      fh_n = 0;
      ff_n = 0;
      if (!kLocal && p == 0) {      // the top border H(0, j) and the F it
        fh_n = V == kVarGlobal ? -gapw(jf + 1, go, ge) : 0;   // feeds into row 1,
        ff_n = fh_n - go;           // max(F(0, j) - ge, H(0, j) - go)
      }
      if (p > 0 && jf < n) {
        const int2 v = rb[jf];
        fh_n = v.x;
        ff_n = v.y;
      }
    };

    int best = kLocal ? 0 : kNegInf;
    int bcol = INT32_MAX, brow = INT32_MAX;   // kEnds: first cell holding `best`
    const int lstar = (a.m - 1) % ROWS / R, kstar = (a.m - 1) % R;   // the last row (modes)
    if (w == 0 && my_rounds > 0) fetch(0, 0);
    for (int T = 0; T < kSkew * w; ++T) {
      if (T == kSkew * w - 1 && my_rounds > 0) fetch(w, 0);
      __syncthreads();
    }
    for (int q = 0; q < my_rounds; ++q) {
      const int p = q * W2 + w;
      const bool more = q + 1 < my_rounds;
      const bool last_pass = p == P - 1;
      {  // stage this pass's profile rows (read back only by this wave)
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(qprof);
        uint4* dst = reinterpret_cast<uint4*>(lprof);
        constexpr int per_code = ROWS / 16;           // uint4 per code row
        const int src_stride = qd.m_pad2 / 16;
        for (int x = lane; x < kIntraCodes * per_code; x += 64) {
          const int code = x / per_code, r = x - code * per_code;
          dst[x] = src[(size_t)code * src_stride + (size_t)p * per_code + r];
        }
        // LDS operations of one wave execute in order; keep the compiler
        // from moving the reads below above these writes
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
      int H[R], E[R];
      const int top = p * ROWS + lane * R;      // rows top + 1 .. top + R (1-based)
#pragma unroll
      for (int k = 0; k < R; ++k) {
        H[k] = kLocal ? 0 : -gapw(top + k + 1, go, ge);   // H(i, 0)
        E[k] = kLocal ? 0 : H[k] - go;                    // E(i, 1)
      }
      int hdiag = kLocal ? 0 : -gapw(top, go, ge), code = SW_PAD_CODE;
      int hbot = H[R - 1], fbot = 0;
      int pbest = 0, pcol = 0, pk = 0;          // kEnds: this pass's first maximum
      for (int c = 0; c < C2; ++c) {
        int fcode = fcode_n, fh = fh_n, ff = ff_n;
        if (c + 1 < C2) fetch(p, c + 1);
        else if (more) fetch(p + W2, 0);
        int collh = 0, collf = 0;
#pragma unroll 2
        for (int tau = 0; tau < 64; ++tau) {
          code = shr_in(code, fcode);
          const int hup = shr_in(hbot, fh);
          const int fup = shr_in(fbot, ff);
          fcode = shl_in(fcode, SW_PAD_CODE);
          fh = shl_in(fh, 0);
          ff = shl_in(ff, 0);
          const PV pv = *reinterpret_cast<const PV*>(lprof + code * ROWS + lane * R);
          int prof[R];
          unpack_profile<R>(pv, prof);
          int hd = hdiag;
          hdiag = hup;
          int F = fup;
          const int col = c * 64 + tau - lane;    // this step's column
          uint32_t tcode[(R + 3) / 4];             // kTrace: this step's codes
#pragma unroll
          for (int x = 0; x < (R + 3) / 4; ++x) tcode[x] = 0;
          if (kLocal || col >= 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
              const int d = hd + prof[k];
              const int h = imax(imax(d, E[k]), F);
              if constexpr (kTrace) {
                const uint32_t src = h == 0 ? 0u : h == d ? 1u : h == F ? 3u : 2u;
                const uint32_t op = (h - go >= E[k] - ge ? 4u : 0u) | (h - go >= F - ge ? 8u : 0u);
                tcode[k >> 2] |= (src | op) << (8 * (k & 3));
              }
              hd = H[k];
              H[k] = h;
              if constexpr (kEnds) {
                if (h > pbest) { pbest = h; pcol = col; pk = k; }
              } else if constexpr (kLocal) {
                best = imax(best, h);
              }
              const int t = h - go;
              if constexpr (kLocal) {
                E[k] = imax(imax(E[k] - ge, t), 0);
                F = imax(imax(F - ge, t), 0);
              } else {
                E[k] = imax(E[k] - ge, t);
                F = imax(F - ge, t);
              }
            }
          }
          if constexpr (kTrace) {
            if (col >= 0 && col < n) {
              uint8_t* at = dir + (size_t)col * a.dir_ld + (size_t)top;
              if constexpr (R == 8) {
                *reinterpret_cast<uint2*>(at) = make_uint2(tcode[0], tcode[1]);
              } else if constexpr (R == 4) {
                *reinterpret_cast<uint32_t*>(at) = tcode[0];
              } else {
                *reinterpret_cast<uint16_t*>(at) = (uint16_t)tcode[0];
              }
            }
          }
          if constexpr (!kLocal) {
            if (last_pass && lane == lstar && col >= 0 && col < n) {
              int v = H[0];
#pragma unroll
              for (int k = 1; k < R; ++k) v = k == kstar ? H[k] : v;
              if (V == kVarGlobal) {
                if (col == n - 1) best = v;
              } else {
                best = imax(best, v);
              }
            }
          }
          hbot = H[R - 1];
          fbot = F;
          collh = shl_in(collh, hbot);
          collf = shl_in(collf, fbot);
        }
        const int jo = c * 64 + lane - 63;
        if (!last_pass && jo >= 0 && jo < n) rb[jo] = make_int2(collh, collf);
        __syncthreads();
      }
      if constexpr (kEnds) {
        const int prow = p * ROWS + lane * R + pk;
        if (pbest > best || (pbest == best && pbest > 0 &&
                             (pcol < bcol || (pcol == bcol && prow < brow)))) {
          best = pbest;
          bcol = pcol;
          brow = prow;
        }
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    for (int T = kSkew * w + my_rounds * C2; T < T_total; ++T) __syncthreads();

    if constexpr (kEnds) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const int ob = __shfl_xor(best, off, 64);
        const int oc = __shfl_xor(bcol, off, 64);
        const int orow = __shfl_xor(brow, off, 64);
        if (end_before(ob, oc, orow, best, bcol, brow)) { best = ob; bcol = oc; brow = orow; }
      }
      if (lane == 0) { lbest[w] = best; lpos[2 * w] = bcol; lpos[2 * w + 1] = brow; }
      __syncthreads();
      if (threadIdx.x == 0) {
        int b = lbest[0], bc = lpos[0], br = lpos[1];
#pragma unroll
        for (int x = 1; x < W2; ++x)
          if (end_before(lbest[x], lpos[2 * x], lpos[2 * x + 1], b, bc, br)) {
            b = lbest[x]; bc = lpos[2 * x]; br = lpos[2 * x + 1];
          }
        a.ends[it] = b > 0 ? make_int4(sid, b, br, bc + c0) : make_int4(sid, 0, -1, -1);
      }
    } else {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) best = imax(best, __shfl_xor(best, off, 64));
      if (lane == 0) lbest[w] = best;
      __syncthreads();
      if (threadIdx.x == 0) {
        int b = lbest[0];
#pragma unroll
        for (int x = 1; x < W2; ++x) b = imax(b, lbest[x]);
        a.out[qd.out_off + sid] = (kLocal || n > 0) ? b : -gapw(a.m, go, ge);
      }
    }
    __syncthreads();
  }
}

template <int RP> struct PairVec;
template <> struct PairVec<1> { typedef uint32_t T; };
template <> struct PairVec<2> { typedef uint2 T; };
template <> struct PairVec<4> { typedef uint4 T; };
__device__ __forceinline__ uint32_t pv_get(const uint32_t& v, int) { return v; }
__device__ __forceinline__ uint32_t pv_get(const uint2& v, int j) { return j ? v.y : v.x; }
__device__ __forceinline__ uint32_t pv_get(const uint4& v, int j) {
  return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w;
}

// Packed variant for the long list of a single search.  The two halves of
// every register hold two database sequences (a, b) of similar length scored
// against the query in binary16, with the cell arithmetic of the inter-task
// kernels (packed16.h, exact below the rescoring limit); the wavefront,
// passes, pass pipeline and boundary rows are those of k_intra_i32, each
// value now carrying both sequences.  The profile is binary16 row pairs
// [code][row/2]: a lane reads R/2 dwords (its R rows) for each sequence's
// residue and one byte permute per row packs the two sequences' scores.  The
// residue codes travel down the wave pre-multiplied into byte offsets of a
// code row, a's in the low and b's in the high 16 bits of one register.
// Sequences whose maximum reaches the limit go to the rescoring list.
template <int R, int W2>
__global__ __launch_bounds__(64 * W2) void k_intra_f16(IntraPairArgs a) {
  constexpr int ROWS = 64 * R;        // query rows per pass
  constexpr int RP = R / 2;           // row-pair dwords per lane and code
  constexpr int CODE_DW = ROWS / 2;   // dwords per code row of a pass
  constexpr uint32_t kCodeBytes = CODE_DW * 4;
  static_assert(SW_PAD_CODE * kCodeBytes < 65536, "code offsets must fit 16 bits");
  constexpr uint32_t kPadPair = (SW_PAD_CODE * kCodeBytes) * 0x10001u;
  typedef typename PairVec<RP>::T PV;
  __shared__ __align__(16) uint32_t lprof_all[W2][kIntraCodes * CODE_DW];
  __shared__ uint32_t lbest[W2];

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* lprof = &lprof_all[w][0];
  const char* lbase = reinterpret_cast<const char*>(lprof) + lane * RP * 4;
  int2* __restrict__ rb = a.scratch + (size_t)blockIdx.x * a.scratch_stride;
  const uint32_t go = a.go2, ge = a.ge2;

  for (int it = blockIdx.x; it < a.count; it += gridDim.x) {
    const int2 seg = a.seg_items ? a.seg_items[it] : make_int2(it, 0);
    // the query: the search's, or (batches) the item's own
    const int2 bitem = a.batch_items ? a.batch_items[it] : make_int2(seg.x, 0);
    const uint32_t* __restrict__ prof3 = a.prof3;
    int m_pad2 = a.m_pad2, P = a.n_pass;
    int64_t out_off = 0;
    if (a.batch_items) {
      const QueryDesc qd = a.queries[bitem.y];
      prof3 += qd.prof3_off;
      m_pad2 = qd.m_pad2;
      P = qd.n_pass3;
      out_off = qd.out_off;
    }
    const int q_last = (P - 1) / W2, w_last = (P - 1) % W2;
    const int my_rounds = (w < P) ? (P - 1 - w) / W2 + 1 : 0;
    const int2 item = a.items[bitem.x];
    const int sa = item.x, sb = item.y;
    const int64_t ba = a.offs[sa];
    int na = (int)(a.offs[sa + 1] - ba);
    const int64_t bb = sb >= 0 ? a.offs[sb] : 0;
    int nb = sb >= 0 ? (int)(a.offs[sb + 1] - bb) : 0;
    const uint8_t* __restrict__ sqa = a.res + ba;
    const uint8_t* __restrict__ sqb = a.res + bb;
    if (a.seg_items) {
      // the segment's window: columns [c0, hi) of both sequences, each cut
      // to its own length (a is the longer one: na = 0 only for two empty
      // sequences, handled below); an empty b points at a's residues so that
      // its clamped reads stay in bounds
      const int lo = seg.y * a.seg_cols;
      const int hi = min(na, lo + a.seg_cols);
      const int c0 = max(0, lo - a.seg_overlap);
      na = hi - c0;
      nb = max(0, min(nb, hi) - c0);
      sqa += c0;
      sqb = nb > 0 ? sqb + c0 : sqa;
    }
    // the item's result from its packed maximum b (thread 0): the
    // segment's maximum, or per half the score or, at the rescoring limit,
    // an entry of the rescoring list
    auto emit = [&](uint32_t b) {
      if (a.seg_best) {
        a.seg_best[it] = b;
        return;
      }
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int sid = half ? sb : sa;
        if (sid < 0) continue;
        const int score = half_score(b, half, a.sat_limit);
        if (score < 0) {
          const int idx = atomicAdd(a.flag_count, 1);
          a.flag_list[idx] = make_int2(sid, bitem.y);
        } else {
          a.out[out_off + sid] = score;
        }
      }
    };
    const int n = na > nb ? na : nb;
    if (n == 0) {
      // two empty sequences (a pair of a handed-over short bin): maximum 0,
      // and no residue or boundary-row read; the whole workgroup skips alike
      if (threadIdx.x == 0) emit(0u);
      continue;
    }
    if (nb == 0) sqb = sqa;   // an empty b reads a's residues (clamped, in bounds)
    const int C2 = max((n + 63 + 63) >> 6, kSkew * W2);
    const int T_total = q_last * C2 + kSkew * w_last + C2;

    // the next chunk's inputs, loaded a chunk ahead: the raw residue bytes
    // and the row above, every load issued (its index clamped into the
    // sequence or the scratch row), the padding chosen and the codes packed
    // where they are used, so no load is waited for before then
    uint32_t ca_n = SW_PAD_CODE, cb_n = SW_PAD_CODE, fh_n = 0, ff_n = 0;
    bool va_n = false, vb_n = false, vr_n = false;
    auto fetch = [&](int p, int c) {
      const int jf = c * 64 + lane;
      ca_n = sqa[min(jf, na - 1)];
      cb_n = sqb[min(jf, max(nb - 1, 0))];
      const int2 v = rb[min(jf, n - 1)];
      fh_n = (uint32_t)v.x;
      ff_n = (uint32_t)v.y;
      va_n = jf < na;
      vb_n = jf < nb;
      vr_n = p > 0 && jf < n;
    };

    uint32_t best = 0;
    if (w == 0 && my_rounds > 0) fetch(0, 0);
    for (int T = 0; T < kSkew * w; ++T) {
      if (T == kSkew * w - 1 && my_rounds > 0) fetch(w, 0);
      __syncthreads();
    }
    for (int q = 0; q < my_rounds; ++q) {
      const int p = q * W2 + w;
      const bool more = q + 1 < my_rounds;
      const bool last_pass = p == P - 1;
      {  // stage this pass's profile row pairs (read back only by this wave)
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(prof3);
        uint4* dst = reinterpret_cast<uint4*>(lprof);
        constexpr int per_code = CODE_DW / 4;          // uint4 per code row
        const int src_stride = m_pad2 / 8;             // uint4 per code in prof3
        for (int x = lane; x < kIntraCodes * per_code; x += 64) {
          const int code = x / per_code, r = x - code * per_code;
          dst[x] = src[(size_t)code * src_stride + (size_t)p * per_code + r];
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
      uint32_t H[R], E[R];
#pragma unroll
      for (int k = 0; k < R; ++k) { H[k] = 0; E[k] = 0; }
      uint32_t hdiag = 0, code = kPadPair, hbot = 0, fbot = 0;
      // nothing pending at the chunk loop's entry: a scalar load pending
      // there (they return out of order) would make every step wait for the
      // next step's profile reads as well as its own
      __builtin_amdgcn_s_waitcnt(0);   // vmcnt(0) expcnt(0) lgkmcnt(0)
      for (int c = 0; c < C2; ++c) {
        uint32_t fcode = (va_n ? ca_n : (uint32_t)SW_PAD_CODE) * kCodeBytes |
                         ((vb_n ? cb_n : (uint32_t)SW_PAD_CODE) * kCodeBytes) << 16;
        uint32_t fh = vr_n ? fh_n : 0, ff = vr_n ? ff_n : 0;
        if (c + 1 < C2) fetch(p, c + 1);
        else if (more) fetch(p + W2, 0);
        uint32_t collh = 0, collf = 0;
        // the codes of step tau + 1 are those of step tau shifted one lane
        // (the inputs shifted in with them), so each step's profile reads are
        // issued a step ahead; the chunk's first step reads at its start.  The
        // extra read after the last step is of a valid code and unused.
        uint32_t code_c = (uint32_t)shr_in((int)code, (int)fcode);
        fcode = (uint32_t)shl_in((int)fcode, (int)kPadPair);
        PV va = *reinterpret_cast<const PV*>(lbase + (code_c & 0xffffu));
        PV vb = *reinterpret_cast<const PV*>(lbase + (code_c >> 16));
#pragma unroll 2
        for (int tau = 0; tau < 64; ++tau) {
          const uint32_t code_n = (uint32_t)shr_in((int)code_c, (int)fcode);
          fcode = (uint32_t)shl_in((int)fcode, (int)kPadPair);
          const PV va_n = *reinterpret_cast<const PV*>(lbase + (code_n & 0xffffu));
          const PV vb_n = *reinterpret_cast<const PV*>(lbase + (code_n >> 16));
          code = code_c;
          const uint32_t hup = (uint32_t)shr_in((int)hbot, (int)fh);
          const uint32_t fup = (uint32_t)shr_in((int)fbot, (int)ff);
          fh = (uint32_t)shl_in((int)fh, 0);
          ff = (uint32_t)shl_in((int)ff, 0);
          uint32_t pr[R];
#pragma unroll
          for (int j = 0; j < RP; ++j) {
            const uint32_t A = pv_get(va, j), B = pv_get(vb, j);
            pr[2 * j] = __builtin_amdgcn_perm(B, A, 0x05040100u);
            pr[2 * j + 1] = __builtin_amdgcn_perm(B, A, 0x07060302u);
          }
          uint32_t hd = hdiag;
          hdiag = hup;
          uint32_t F = fup;
          uint32_t hprev = 0;
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const uint32_t h = cell(hd, H[k], E[k], F, pr[k], go, ge);
            if (k & 1) best = hmax3(best, hprev, h);
            else hprev = h;
          }
          hbot = H[R - 1];
          fbot = F;
          collh = (uint32_t)shl_in((int)collh, (int)hbot);
          collf = (uint32_t)shl_in((int)collf, (int)fbot);
          code_c = code_n;
          va = va_n;
          vb = vb_n;
        }
        const int jo = c * 64 + lane - 63;
        if (!last_pass && jo >= 0 && jo < n) rb[jo] = make_int2((int)collh, (int)collf);
        __syncthreads();
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    for (int T = kSkew * w + my_rounds * C2; T < T_total; ++T) __syncthreads();

#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = hmax2(best, (uint32_t)__shfl_xor((int)best, off, 64));
    if (lane == 0) lbest[w] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t b = lbest[0];
#pragma unroll
      for (int x = 1; x < W2; ++x) b = hmax2(b, lbest[x]);
      emit(b);
    }
    __syncthreads();
  }
}

// The score of each segmented pair: the maximum over its segments' packed
// maxima (each a lower bound of the pair's scores, and the segment holding a
// sequence's best cell computes that cell exactly), then per half the score
// or, at the rescoring limit, an entry of the rescoring list.
__global__ void k_long_combine(const int2* __restrict__ pairs, const int32_t* __restrict__ seg0,
                               int32_t n_pairs, const uint32_t* __restrict__ seg_best,
                               int32_t sat_limit, int32_t* __restrict__ out,
                               int32_t* flag_count, int2* __restrict__ flag_list) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  uint32_t b = 0;
  for (int x = seg0[p]; x < seg0[p + 1]; ++x) b = hmax2(b, seg_best[x]);
  const int2 item = pairs[p];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int sid = half ? item.y : item.x;
    if (sid < 0) continue;
    const int score = half_score(b, half, sat_limit);
    if (score < 0) {
      const int idx = atomicAdd(flag_count, 1);
      flag_list[idx] = make_int2(sid, 0);
    } else {
      out[sid] = score;
    }
  }
}

template <int R, int W2>
hipError_t launch_pair_rw(int grid, const IntraPairArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_intra_f16<R, W2>), dim3(grid), dim3(64 * W2), 0, s, a);
  return hipGetLastError();
}

template <int R, int W2>
hipError_t launch_rw(int grid, const IntraArgs& a, hipStream_t s) {
  if (a.mode == SW_MODE_GLOBAL)
    hipLaunchKernelGGL((k_intra_i32<R, W2, kVarGlobal>), dim3(grid), dim3(64 * W2), 0, s, a);
  else if (a.mode == SW_MODE_SEMIGLOBAL)
    hipLaunchKernelGGL((k_intra_i32<R, W2, kVarSemi>), dim3(grid), dim3(64 * W2), 0, s, a);
  else if (a.ends && a.dir)
    hipLaunchKernelGGL((k_intra_i32<R, W2, kVarTrace>), dim3(grid), dim3(64 * W2), 0, s, a);
  else if (a.ends)
    hipLaunchKernelGGL((k_intra_i32<R, W2, kVarEnds>), dim3(grid), dim3(64 * W2), 0, s, a);
  else
    hipLaunchKernelGGL((k_intra_i32<R, W2, kVarScore>), dim3(grid), dim3(64 * W2), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_intra(int R, int W2, int grid, const IntraArgs& a, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define SWDB_CASE(r, w) \
  if (R == r && W2 == w) return launch_rw<r, w>(grid, a, s);
  SWDB_CASE(2, 1) SWDB_CASE(4, 1) SWDB_CASE(8, 1)
  SWDB_CASE(2, 2) SWDB_CASE(4, 2) SWDB_CASE(8, 2)
  SWDB_CASE(2, 4) SWDB_CASE(4, 4) SWDB_CASE(8, 4)
  SWDB_CASE(2, 8) SWDB_CASE(4, 8) SWDB_CASE(8, 8)
#undef SWDB_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_long_combine(const int2* pairs, const int32_t* seg0, int32_t n_pairs,
                               const uint32_t* seg_best, int32_t sat_limit, int32_t* out,
                               int32_t* flag_count, int2* flag_list, hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_long_combine, dim3((n_pairs + 255) / 256), dim3(256), 0, s, pairs, seg0,
                     n_pairs, seg_best, sat_limit, out, flag_count, flag_list);
  return hipGetLastError();
}

hipError_t launch_intra_pairs(int R, int W2, int grid, const IntraPairArgs& a, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define SWDB_CASE(r, w) \
  if (R == r && W2 == w) return launch_pair_rw<r, w>(grid, a, s);
  SWDB_CASE(2, 1) SWDB_CASE(4, 1) SWDB_CASE(8, 1)
  SWDB_CASE(2, 2) SWDB_CASE(4, 2) SWDB_CASE(8, 2)
  SWDB_CASE(2, 4) SWDB_CASE(4, 4) SWDB_CASE(8, 4)
  SWDB_CASE(2, 8) SWDB_CASE(4, 8)
#undef SWDB_CASE
  return hipErrorInvalidValue;
}

}  // namespace swdb
