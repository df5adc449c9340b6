// Small helper kernels: query profile construction and buffer fill.
#include "internal.h"

namespace swdb {
namespace {

__device__ __forceinline__ int profile_score(const uint8_t* __restrict__ q, int m,
                                             const Matrix& mat, int i, int c) {
  if (i >= m || c >= SW_ALPHA) return kPadScore;
  const int qc = q[i];
  return qc < SW_ALPHA ? (int)mat.v[qc * SW_ALPHA + c] : kPadScore;
}

// Builds the query profiles from the query codes and the substitution
// matrix: the inter-task layout for strips of R rows (see prof_strip_dwords),
// the intra-task layout [25][m_pad2] int8 and, when prof3 is given, the
// packed intra-task layout [25][m_pad2 / 2] of binary16 row pairs (dword
// (c, r) = S(a_2r, c) low, S(a_2r+1, c) high); codes 0..23 and the pad code.
// Entry (i, c) is S(a_i, c); rows past the query end and the pad/spare codes
// get kPadScore.  Thread 0 also clears the rescoring list's count.
__global__ void k_profile(const uint8_t* __restrict__ q, int m, Matrix mat,
                          uint32_t* __restrict__ prof, int m_pad, int R,
                          int8_t* __restrict__ prof2, uint32_t* __restrict__ prof3, int m_pad2,
                          int32_t* __restrict__ flag_count) {
  const int64_t n1 = (int64_t)(m_pad / R) * prof_strip_dwords(R);
  const int64_t n2 = (int64_t)kIntraCodes * m_pad2;
  const int64_t n3 = prof3 ? (int64_t)kIntraCodes * (m_pad2 / 2) : 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0 && flag_count) *flag_count = 0;
  for (; idx < n1 + n2 + n3; idx += stride) {
    if (idx < n1) {
      // idx = ((strip * 2 + table) * R / 2 + pair) * kProfPairDwords + 2 * c + t
      const int rem = (int)(idx % kProfPairDwords);
      const int64_t pr = idx / kProfPairDwords;
      const int pair = (int)(pr % (R / 2));
      const int64_t st = pr / (R / 2);
      const int i = (int)(st >> 1) * R + 2 * pair + (rem & 1), c = rem >> 1;
      const uint32_t v = half_bits(profile_score(q, m, mat, i, c));
      prof[idx] = (st & 1) ? kHalfOne | (v << 16) : v | (kHalfOne << 16);
    } else if (idx < n1 + n2) {
      const int64_t j = idx - n1;
      const int c = (int)(j / m_pad2), i = (int)(j % m_pad2);
      prof2[j] = (int8_t)profile_score(q, m, mat, i, c);
    } else {
      const int64_t j = idx - n1 - n2;
      const int half_rows = m_pad2 / 2;
      const int c = (int)(j / half_rows), r = (int)(j % half_rows);
      const uint32_t lo = half_bits(profile_score(q, m, mat, 2 * r, c));
      const uint32_t hi = half_bits(profile_score(q, m, mat, 2 * r + 1, c));
      prof3[j] = lo | (hi << 16);
    }
  }
}

// Pair profiles and intra-task profiles of a batch.  blockIdx.y < n_pairs
// selects a pair: the dword of row i and code c of its profile (n_strips * R
// rows in the kProfRowDwords layout) holds (S(a_i, c), S(b_i, c)) as
// binary16, kPadScore past either query's end.  Larger
// blockIdx.y select a query's intra-task [25][m_pad2] int8 profile and, when
// prof3 is given, its packed [25][m_pad2 / 2] binary16 row pairs.
__global__ void k_batch_profiles(const uint8_t* __restrict__ queries,
                                 const int64_t* __restrict__ qoffs, Matrix mat,
                                 const PairDesc* __restrict__ pairs, int n_pairs, int R,
                                 uint32_t* __restrict__ prof,
                                 const QueryDesc* __restrict__ qdesc, int8_t* __restrict__ prof2,
                                 uint32_t* __restrict__ prof3) {
  const int y = blockIdx.y;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (y < n_pairs) {
    const PairDesc pd = pairs[y];
    const int64_t total = (int64_t)pd.n_strips * R * kBatchRowDwords;
    const uint8_t* qa = queries + qoffs[pd.qa];
    const int ma = (int)(qoffs[pd.qa + 1] - qoffs[pd.qa]);
    const uint8_t* qb = pd.qb >= 0 ? queries + qoffs[pd.qb] : nullptr;
    const int mb = pd.qb >= 0 ? (int)(qoffs[pd.qb + 1] - qoffs[pd.qb]) : 0;
    for (int64_t idx = start; idx < total; idx += stride) {
      const int rem = (int)(idx % kProfPairDwords);
      const int i = 2 * (int)(idx / kProfPairDwords) + (rem & 1), c = rem >> 1;
      const uint32_t lo = half_bits(profile_score(qa, ma, mat, i, c));
      const uint32_t hi = half_bits(profile_score(qb, mb, mat, i, c));
      prof[pd.prof_off + idx] = lo | (hi << 16);
    }
  } else {
    const int qi = y - n_pairs;
    const QueryDesc qd = qdesc[qi];
    const uint8_t* q = queries + qoffs[qi];
    const int m = (int)(qoffs[qi + 1] - qoffs[qi]);
    const int64_t total = (int64_t)kIntraCodes * qd.m_pad2;
    for (int64_t idx = start; idx < total; idx += stride) {
      const int c = (int)(idx / qd.m_pad2), i = (int)(idx % qd.m_pad2);
      prof2[qd.prof2_off + idx] = (int8_t)profile_score(q, m, mat, i, c);
    }
    if (prof3) {   // packed binary16 row pairs [25][m_pad2 / 2] (the layout of k_profile)
      const int half_rows = qd.m_pad2 / 2;
      for (int64_t idx = start; idx < (int64_t)kIntraCodes * half_rows; idx += stride) {
        const int c = (int)(idx / half_rows), r = (int)(idx % half_rows);
        const uint32_t lo = half_bits(profile_score(q, m, mat, 2 * r, c));
        const uint32_t hi = half_bits(profile_score(q, m, mat, 2 * r + 1, c));
        prof3[qd.prof3_off + idx] = lo | (hi << 16);
      }
    }
  }
}

__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

}  // namespace

hipError_t launch_profile(const uint8_t* d_query, int m, const Matrix& mat, uint32_t* prof,
                          int m_pad, int R, int8_t* prof2, uint32_t* prof3, int m_pad2,
                          int32_t* flag_count, hipStream_t s) {
  if (R <= 0 || R % 2 != 0 || m_pad % R != 0) return hipErrorInvalidValue;
  const int64_t total = (int64_t)(m_pad / R) * prof_strip_dwords(R) +
                        (int64_t)kIntraCodes * m_pad2 +
                        (prof3 ? (int64_t)kIntraCodes * (m_pad2 / 2) : 0);
  int grid = (int)std::min<int64_t>((total + 255) / 256, 2048);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_profile, dim3(grid), dim3(256), 0, s, d_query, m, mat, prof, m_pad, R,
                     prof2, prof3, m_pad2, flag_count);
  return hipGetLastError();
}

hipError_t launch_batch_profiles(const uint8_t* d_queries, const int64_t* d_qoffs, int n_queries,
                                 const Matrix& mat, const PairDesc* d_pairs, int n_pairs, int R,
                                 int64_t max_work, uint32_t* prof, const QueryDesc* d_qdesc,
                                 int8_t* prof2, uint32_t* prof3, hipStream_t s) {
  const int ys = n_pairs + n_queries;
  if (ys <= 0) return hipSuccess;
  if (ys > 65535) return hipErrorInvalidValue;
  const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((max_work + 255) / 256, 256));
  hipLaunchKernelGGL(k_batch_profiles, dim3(gx, ys), dim3(256), 0, s, d_queries, d_qoffs, mat,
                     d_pairs, n_pairs, R, prof, d_qdesc, prof2, prof3);
  return hipGetLastError();
}

hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace swdb
