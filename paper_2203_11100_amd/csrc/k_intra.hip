// Intra-task Smith-Waterman/Gotoh kernel for long database sequences and for
// exact 32-bit rescoring (paper section 2.2: intra-task parallelism, all
// processing elements work on one alignment matrix and neighbours exchange
// border elements; section 2.3: SW#db switches to it by sequence length).
//
// One wave scores one (query, database sequence) pair.  Lane l owns R
// consecutive query rows of the current pass (a pass covers 64*R rows) and
// the wave sweeps the database sequence as an anti-diagonal wavefront: at
// step t lane l computes column j = t - l of its rows, so lane l receives the
// H and F values of row (top - 1) for column j from lane l-1, which computed
// them in the previous step.  The exchange is one cross-lane DPP move per
// value (wave_shr:1); no LDS and no barrier are needed inside the wave.
// Lane 0 takes its inputs from the previous pass's bottom row (kept in a
// per-workgroup global buffer), and the last lane's bottom row is collected
// for the next pass; residue codes and the boundary row are fed in 64
// columns at a time and shifted down the wave one lane per step.
//
// Cells use the exact recurrence in 32-bit integers, E and F kept as
// max(E, 0) and max(F, 0) (equivalent because H >= 0; see the inter-task
// kernel), so H = max(H_diag + S, E, F) is one three-input maximum.
// Columns before a lane's first column and after the sequence's end see the
// pad code, whose profile score is <= 0, so they never raise the maximum.
//
// The pass's profile is staged in LDS as [code][row]: lanes read their R rows
// for their own residue code, R*2 contiguous bytes at code*64R*2 + 2Rl, which
// keeps the 64 reads of a wave in distinct banks whatever the codes are.
#include "internal.h"

namespace swdb {
namespace {

constexpr int kWaveShr1 = 0x138;  // DPP wave_shr:1  (lane l <- lane l-1)
constexpr int kWaveShl1 = 0x130;  // DPP wave_shl:1  (lane l <- lane l+1)

// lane l <- lane l-1; lane 0 keeps `first`
__device__ __forceinline__ int shr_in(int v, int first) {
  return __builtin_amdgcn_update_dpp(first, v, kWaveShr1, 0xf, 0xf, false);
}
// lane l <- lane l+1; lane 63 keeps `last`
__device__ __forceinline__ int shl_in(int v, int last) {
  return __builtin_amdgcn_update_dpp(last, v, kWaveShl1, 0xf, 0xf, false);
}

template <int R> struct ProfVec;
template <> struct ProfVec<2> { typedef uint32_t T; };
template <> struct ProfVec<4> { typedef uint2 T; };
template <> struct ProfVec<8> { typedef uint4 T; };

template <int R>
__device__ __forceinline__ void unpack_profile(const typename ProfVec<R>::T& v, int (&p)[R]);
template <>
__device__ __forceinline__ void unpack_profile<2>(const uint32_t& v, int (&p)[2]) {
  p[0] = (int)(short)(v & 0xffffu);
  p[1] = (int)v >> 16;
}
template <>
__device__ __forceinline__ void unpack_profile<4>(const uint2& v, int (&p)[4]) {
  p[0] = (int)(short)(v.x & 0xffffu); p[1] = (int)v.x >> 16;
  p[2] = (int)(short)(v.y & 0xffffu); p[3] = (int)v.y >> 16;
}
template <>
__device__ __forceinline__ void unpack_profile<8>(const uint4& v, int (&p)[8]) {
  p[0] = (int)(short)(v.x & 0xffffu); p[1] = (int)v.x >> 16;
  p[2] = (int)(short)(v.y & 0xffffu); p[3] = (int)v.y >> 16;
  p[4] = (int)(short)(v.z & 0xffffu); p[5] = (int)v.z >> 16;
  p[6] = (int)(short)(v.w & 0xffffu); p[7] = (int)v.w >> 16;
}

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

template <int R>
__global__ __launch_bounds__(64) void k_intra_i32(IntraArgs a) {
  constexpr int ROWS = 64 * R;                 // query rows per pass
  extern __shared__ __align__(16) int16_t lprof[];   // [kIntraCodes][ROWS]
  typedef typename ProfVec<R>::T PV;

  const int lane = threadIdx.x;
  const int count = a.count_ptr ? *a.count_ptr : a.count;
  int2* __restrict__ rb = a.scratch + (size_t)blockIdx.x * a.scratch_stride;
  const int go = a.go, ge = a.ge;

  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const int sid = a.items[it];
    const int64_t b0 = a.offs[sid];
    const int n = (int)(a.offs[sid + 1] - b0);
    const uint8_t* __restrict__ bseq = a.res + b0;
    int best = 0;
    const int n_super = (n + 63 + 63) >> 6;   // steps n + 63, 64 per superstep
    for (int p = 0; p < a.n_pass; ++p) {
      __syncthreads();   // the previous pass is done reading lprof
      {
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(a.prof2);
        uint4* dst = reinterpret_cast<uint4*>(lprof);
        const int per_code = ROWS / 8;         // uint4 per code row
        const int src_stride = a.m_pad2 / 8;
        for (int x = lane; x < kIntraCodes * per_code; x += 64) {
          const int code = x / per_code, r = x - code * per_code;
          dst[x] = src[(size_t)code * src_stride + (size_t)p * per_code + r];
        }
      }
      __syncthreads();
      const bool last_pass = (p == a.n_pass - 1);
      const bool first_pass = (p == 0);
      int H[R], E[R];
#pragma unroll
      for (int k = 0; k < R; ++k) { H[k] = 0; E[k] = 0; }
      int hdiag = 0, code = SW_PAD_CODE, hbot = 0, fbot = 0;
      for (int c = 0; c < n_super; ++c) {
        const int jf = c * 64 + lane;
        int fcode = jf < n ? (int)bseq[jf] : SW_PAD_CODE;
        int fh = 0, ff = 0;
        if (!first_pass && jf < n) { const int2 v = rb[jf]; fh = v.x; ff = v.y; }
        int collh = 0, collf = 0;
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
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const int h = imax(imax(hd + prof[k], E[k]), F);
            hd = H[k];
            H[k] = h;
            best = imax(best, h);
            const int t = h - go;
            E[k] = imax(imax(E[k] - ge, t), 0);
            F = imax(imax(F - ge, t), 0);
          }
          hbot = H[R - 1];
          fbot = F;
          collh = shl_in(collh, hbot);
          collf = shl_in(collf, fbot);
        }
        const int jo = c * 64 + lane - 63;
        if (!last_pass && jo >= 0 && jo < n) rb[jo] = make_int2(collh, collf);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = imax(best, __shfl_xor(best, off, 64));
    if (lane == 0) a.out[sid] = best;
  }
}

template <int R>
hipError_t launch_r(int grid, const IntraArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_intra_i32<R>), dim3(grid), dim3(64), intra_lds_bytes(R), s, a);
  return hipGetLastError();
}

}  // namespace

int intra_lds_bytes(int R) { return kIntraCodes * 64 * R * (int)sizeof(int16_t); }

hipError_t launch_intra(int R, int grid, const IntraArgs& a, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (R == 2) return launch_r<2>(grid, a, s);
  if (R == 4) return launch_r<4>(grid, a, s);
  if (R == 8) return launch_r<8>(grid, a, s);
  return hipErrorInvalidValue;
}

}  // namespace swdb
