// Device top-k over one row of scores: the k best database sequences of a
// search, ordered by score (highest first) and, among equal scores, by
// sequence index (smallest first).  SW# reports the best hits of a search
// and their alignments, not only per-sequence scores (paper section 2.3);
// the end coordinates of each hit's best alignment are then computed by the
// exact 32-bit intra-task kernel over these k sequences only.
//
// Selection is a most-significant-digit radix select on order-preserving
// 32-bit keys (the score with its sign bit flipped), 8 bits per pass: each
// pass histograms the keys that agree with the digits fixed so far, and the
// last workgroup to finish the pass (a ticket counter) picks the digit at
// which the count from the top reaches the number still needed.  After four
// passes the threshold key T is exact, together with `need`, how many
// sequences of key T belong to the top k (the smallest indices among them).
// A counting pass and an ordered compaction then collect every sequence
// above T (in any order) and the first `need` of key T (in index order), and
// one workgroup sorts the k candidates with a bitonic network in LDS.  All
// passes read the score row with coalesced grid-stride or chunked loops;
// every buffer is sized by the host (k <= SW_MAX_TOPK).
#include <algorithm>

#include "internal.h"

namespace swdb {
namespace {

constexpr int kSelThreads = 256;
constexpr int kSortThreads = 1024;

__device__ __forceinline__ uint32_t score_key(int32_t s) { return (uint32_t)s ^ 0x80000000u; }

// Clears the selection state: no digits fixed, `need` = k.
__global__ void k_topk_init(TopkState* st, int32_t k) {
  const int t = threadIdx.x;
  st->hist[t] = 0;
  if (t == 0) {
    st->prefix = 0;
    st->need = k;
    st->done = 0;
    st->n_gt = 0;
  }
}

// One radix pass over bits [shift, shift + 8) of the keys whose higher bits
// equal the prefix fixed by earlier passes.
__global__ __launch_bounds__(kSelThreads) void k_topk_pass(const int32_t* __restrict__ scores,
                                                           int64_t n, TopkState* st, int shift) {
  __shared__ uint32_t h[256];
  __shared__ uint32_t ticket;
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const uint32_t prefix = st->prefix;
  const uint32_t hi_mask = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
  const int64_t stride = (int64_t)gridDim.x * kSelThreads;
  for (int64_t i = (int64_t)blockIdx.x * kSelThreads + t; i < n; i += stride) {
    const uint32_t key = score_key(scores[i]);
    if ((key & hi_mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[t]) atomicAdd(&st->hist[t], h[t]);
  __threadfence();
  __syncthreads();
  if (t == 0) ticket = atomicAdd(&st->done, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return;
  // the last workgroup of the pass: every other workgroup's counts are in
  // st->hist (device-scope atomics, made visible by their fences)
  __threadfence();
  const uint32_t c = __hip_atomic_load(&st->hist[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // count of keys with a digit above t: exclusive suffix sum over the digits
  h[t] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t v = t + off < 256 ? h[t + off] : 0u;
    __syncthreads();
    h[t] += v;
    __syncthreads();
  }
  const uint32_t incl = h[t];          // keys with digit >= t
  const uint32_t above = incl - c;     // keys with digit > t
  const uint32_t need = (uint32_t)st->need;
  __syncthreads();
  if (above < need && incl >= need) {  // exactly one digit satisfies this
    st->prefix = prefix | ((uint32_t)t << shift);
    st->need = (int32_t)(need - above);
  }
  st->hist[t] = 0;
  if (t == 0) st->done = 0;
}

// Chunk of the score row owned by workgroup b in the two ordered passes.
__device__ __forceinline__ void chunk_of(int64_t n, int b, int nb, int64_t* lo, int64_t* hi) {
  const int64_t per = ((n + nb - 1) / nb + kSelThreads - 1) / kSelThreads * kSelThreads;
  *lo = min<int64_t>(n, (int64_t)b * per);
  *hi = min<int64_t>(n, *lo + per);
}

// Per-workgroup count of keys equal to the threshold.
__global__ __launch_bounds__(kSelThreads) void k_topk_count(const int32_t* __restrict__ scores,
                                                            int64_t n, TopkState* st) {
  __shared__ int32_t part[kSelThreads / 64];
  const int t = threadIdx.x;
  const uint32_t T = st->prefix;
  int64_t lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  int32_t c = 0;
  for (int64_t i = lo + t; i < hi; i += kSelThreads) c += score_key(scores[i]) == T;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((t & 63) == 0) part[t >> 6] = c;
  __syncthreads();
  if (t == 0) {
    int32_t s = 0;
#pragma unroll
    for (int x = 0; x < kSelThreads / 64; ++x) s += part[x];
    st->blockcnt[blockIdx.x] = s;
  }
}

// Collects the sequences above the threshold (any order, through a counter)
// and the first `need` sequences equal to it (index order: each workgroup
// ranks its chunk's equal keys after those of the workgroups before it).
__global__ __launch_bounds__(kSelThreads) void k_topk_collect(const int32_t* __restrict__ scores,
                                                              int64_t n, TopkState* st,
                                                              int32_t* __restrict__ gt,
                                                              int32_t* __restrict__ ties) {
  __shared__ int32_t part[kSelThreads / 64];
  __shared__ int32_t scan[kSelThreads];
  const int t = threadIdx.x;
  const uint32_t T = st->prefix;
  const int32_t need = st->need;
  // equal keys in the chunks before this one
  int32_t base = 0;
  for (int x = t; x < (int)blockIdx.x; x += kSelThreads) base += st->blockcnt[x];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) base += __shfl_xor(base, off, 64);
  if ((t & 63) == 0) part[t >> 6] = base;
  __syncthreads();
  base = 0;
#pragma unroll
  for (int x = 0; x < kSelThreads / 64; ++x) base += part[x];
  int64_t lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  for (int64_t i0 = lo; i0 < hi; i0 += kSelThreads) {   // uniform trip count
    const int64_t i = i0 + t;
    const uint32_t key = i < hi ? score_key(scores[i]) : 0u;
    const bool eq = i < hi && key == T;
    if (i < hi && key > T) gt[atomicAdd(&st->n_gt, 1)] = (int32_t)i;
    // inclusive scan of the equal flags over the tile
    scan[t] = eq ? 1 : 0;
    __syncthreads();
    for (int off = 1; off < kSelThreads; off <<= 1) {
      const int32_t v = t >= off ? scan[t - off] : 0;
      __syncthreads();
      scan[t] += v;
      __syncthreads();
    }
    const int32_t rank = base + scan[t] - (eq ? 1 : 0);
    if (eq && rank < need) ties[rank] = (int32_t)i;
    base += scan[kSelThreads - 1];
    __syncthreads();
  }
}

// Sorts the k candidates (gt[0 .. k - need) then ties[0 .. need)) by
// (score descending, index ascending) and writes the hit list's items
// {sequence, 0} for the end-coordinate kernel.
__global__ __launch_bounds__(kSortThreads) void k_topk_sort(const int32_t* __restrict__ scores,
                                                            const TopkState* st,
                                                            const int32_t* __restrict__ gt,
                                                            const int32_t* __restrict__ ties,
                                                            int32_t k, int2* __restrict__ items) {
  __shared__ uint32_t key[SW_MAX_TOPK];
  __shared__ int32_t idx[SW_MAX_TOPK];
  const int t = threadIdx.x;
  const int n_gt = k - st->need;
  int P = 1;
  while (P < k) P <<= 1;
  for (int x = t; x < P; x += kSortThreads) {
    int32_t id = INT32_MAX;
    uint32_t kv = 0;
    if (x < k) {
      id = x < n_gt ? gt[x] : ties[x - n_gt];
      kv = score_key(scores[id]);
    }
    key[x] = kv;
    idx[x] = id;
  }
  __syncthreads();
  // bitonic sort into "before" order: higher key first, then smaller index
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int x = t; x < P; x += kSortThreads) {
        const int y = x ^ stride;
        if (y > x) {
          const bool up = (x & size) == 0;
          const uint32_t kx = key[x], ky = key[y];
          const int32_t ix = idx[x], iy = idx[y];
          const bool y_first = ky > kx || (ky == kx && iy < ix);
          if (y_first == up) {
            key[x] = ky; key[y] = kx;
            idx[x] = iy; idx[y] = ix;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int x = t; x < k; x += kSortThreads) items[x] = make_int2(idx[x], 0);
}

// Column segments of the hit sequences for the end pass of a short query:
// hit t of length n_t gets max(1, ceil(n_t / C)) items {t, s}, computed over
// the windows of the long-pair kernel's column segments (each exact in its
// own columns); seg0[t] is hit t's first item and seg0[k] the total, which
// the end pass reads on the device.  One workgroup: the counts and their
// exclusive scan in LDS (k <= SW_MAX_TOPK), then every hit's items.
__global__ __launch_bounds__(1024) void k_hit_segments(const int2* __restrict__ items, int32_t k,
                                                       const int64_t* __restrict__ offs, int32_t C,
                                                       int32_t cap, int32_t* __restrict__ seg0,
                                                       int2* __restrict__ seg_items) {
  __shared__ int32_t first[SW_MAX_TOPK + 1];
  const int t0 = threadIdx.x;
  for (int t = t0; t < k; t += 1024) {
    const int sid = items[t].x;
    const int64_t n = offs[sid + 1] - offs[sid];
    const int64_t c = (n + C - 1) / C;
    first[t] = c > 1 ? (int32_t)c : 1;
  }
  __syncthreads();
  if (t0 == 0) {
    int32_t acc = 0;
    for (int t = 0; t < k; ++t) {
      const int32_t c = first[t];
      first[t] = acc;
      acc += c;
    }
    first[k] = acc < cap ? acc : cap;
  }
  __syncthreads();
  for (int t = t0; t <= k; t += 1024) seg0[t] = first[t];
  for (int t = t0; t < k; t += 1024) {
    const int32_t end = t + 1 < k ? first[t + 1] : first[k];
    for (int32_t x = first[t]; x < end && x < cap; ++x) seg_items[x] = make_int2(t, x - first[t]);
  }
}

// Each hit's end from its segments' {sid, score, query end, db end}: the
// highest score, then the smallest database position, then the smallest
// query position; (-1, -1) for a score of 0.
__global__ void k_hit_combine(const int2* __restrict__ items, int32_t k,
                              const int32_t* __restrict__ seg0, const int4* __restrict__ seg_ends,
                              int4* __restrict__ hits) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k) return;
  int b = 0, bc = INT32_MAX, br = INT32_MAX;
  for (int32_t x = seg0[t]; x < seg0[t + 1]; ++x) {
    const int4 e = seg_ends[x];
    if (e.y > b || (e.y == b && e.y > 0 && (e.w < bc || (e.w == bc && e.z < br)))) {
      b = e.y;
      bc = e.w;
      br = e.z;
    }
  }
  hits[t] = b > 0 ? make_int4(items[t].x, b, br, bc) : make_int4(items[t].x, 0, -1, -1);
}

__global__ void k_empty_hits(const int2* __restrict__ items, int32_t k, int4* __restrict__ hits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) hits[i] = make_int4(items[i].x, 0, -1, -1);
}

}  // namespace

static int topk_select_grid(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + 4095) / 4096, kTopkMaxBlocks));
}

hipError_t launch_topk(const int32_t* scores, int64_t n, int32_t k, TopkState* st, int32_t* gt,
                       int32_t* ties, int2* items, hipStream_t s) {
  if (k <= 0 || n <= 0) return hipSuccess;
  if (k > SW_MAX_TOPK || k > n) return hipErrorInvalidValue;
  const int grid = topk_select_grid(n);
  hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, s, st, k);
  for (int shift = 24; shift >= 0; shift -= 8)
    hipLaunchKernelGGL(k_topk_pass, dim3(grid), dim3(kSelThreads), 0, s, scores, n, st, shift);
  hipLaunchKernelGGL(k_topk_count, dim3(grid), dim3(kSelThreads), 0, s, scores, n, st);
  hipLaunchKernelGGL(k_topk_collect, dim3(grid), dim3(kSelThreads), 0, s, scores, n, st, gt, ties);
  hipLaunchKernelGGL(k_topk_sort, dim3(1), dim3(kSortThreads), 0, s, scores, st, gt, ties, k,
                     items);
  return hipGetLastError();
}

hipError_t launch_hit_segments(const int2* items, int32_t k, const int64_t* offs, int32_t C,
                               int32_t cap, int32_t* seg0, int2* seg_items, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (k > SW_MAX_TOPK || C <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hit_segments, dim3(1), dim3(1024), 0, s, items, k, offs, C, cap, seg0,
                     seg_items);
  return hipGetLastError();
}

hipError_t launch_hit_combine(const int2* items, int32_t k, const int32_t* seg0,
                              const int4* seg_ends, int4* hits, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hit_combine, dim3((k + 255) / 256), dim3(256), 0, s, items, k, seg0,
                     seg_ends, hits);
  return hipGetLastError();
}

hipError_t launch_empty_hits(const int2* items, int32_t k, int4* hits, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_empty_hits, dim3((k + 255) / 256), dim3(256), 0, s, items, k, hits);
  return hipGetLastError();
}

}  // namespace swdb
