// Host (CPU) local alignment scorer of the hybrid search.
//
// One database sequence at a time against the query, with Farrar's striped
// SIMD form of Gotoh's recurrence (Farrar 2007): 16 lanes of 16-bit
// integers, lane k of segment s holding query row k * seg + s, so a column
// of the matrix is seg vectors whose only dependency across lanes is the
// vertical gap F.  Each column is computed once with F carried within the
// segments, then F is propagated across lanes in a correction loop that
// stops as soon as it can no longer raise any H (the "lazy F" loop).  The
// correction also raises the next column's E wherever it raises an H, which
// keeps E exact; the scores would not need it (a vertical gap followed by a
// horizontal one costs what the two in the other order cost, and that order
// is in the recurrence already - Farrar's argument).  H, E
// and F are kept at or above 0 (exact for local scores, H >= 0), adds
// saturate at 32767, and a sequence whose maximum reaches 32767 is rescored
// with the scalar recurrence in 32-bit integers - the same saturation
// argument as the packed GPU kernels.  Gap penalties above 32767 act like
// 32767 in 16 bits: with every H below 32767, H - gap is negative either way
// and the floor takes it to 0.
#include "cpu_scorer.h"

#include <string.h>

#include <algorithm>

namespace swdb {
namespace cpu {
namespace {

typedef int16_t v16 __attribute__((ext_vector_type(16)));
typedef v16 v16u __attribute__((aligned(2)));   // unaligned loads and stores

constexpr int kLanes = 16;
constexpr int kCodes = 25;        // residue codes 0..23 and the pad code
constexpr int kPad = 24;
constexpr int16_t kPadScore = -64;
constexpr int16_t kSat = 32767;

inline v16 ld(const int16_t* p) { return *reinterpret_cast<const v16u*>(p); }
inline void st(int16_t* p, v16 v) { *reinterpret_cast<v16u*>(p) = v; }
inline v16 splat(int16_t x) { return (v16)x; }

// lane k <- lane k-1, lane 0 <- 0
inline v16 shift_up(v16 v) {
  const v16 z = splat(0);
  return __builtin_shufflevector(z, v, 0, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28,
                                 29, 30);
}

inline bool any_gt(v16 a, v16 b) { return __builtin_reduce_or(a > b) != 0; }

// The striped kernel; returns the score, or -1 when a 16-bit value saturated.
__attribute__((always_inline)) inline int32_t striped(const Profile& p, const uint8_t* seq, int n,
                                                      int32_t go, int32_t ge, Workspace* w) {
  const int seg = p.seg;
  const v16 zero = splat(0);
  const v16 vgo = splat((int16_t)std::min<int32_t>(go, kSat));
  const v16 vge = splat((int16_t)std::min<int32_t>(ge, kSat));
  int16_t* hl = w->h0.data();
  int16_t* hs = w->h1.data();
  int16_t* ev = w->e.data();
  for (int x = 0; x < seg * kLanes; ++x) hl[x] = hs[x] = ev[x] = 0;
  v16 vmax = zero;
  for (int j = 0; j < n; ++j) {
    const int16_t* prof = p.v.data() + (size_t)seq[j] * seg * kLanes;
    v16 vf = zero;
    v16 vh = shift_up(ld(hl + (seg - 1) * kLanes));     // H(i-1, j-1) entering segment 0
    for (int s = 0; s < seg; ++s) {
      vh = __builtin_elementwise_add_sat(vh, ld(prof + s * kLanes));
      const v16 e = ld(ev + s * kLanes);
      vh = __builtin_elementwise_max(__builtin_elementwise_max(vh, e),
                                     __builtin_elementwise_max(vf, zero));
      vmax = __builtin_elementwise_max(vmax, vh);
      st(hs + s * kLanes, vh);
      const v16 t = __builtin_elementwise_sub_sat(vh, vgo);
      st(ev + s * kLanes, __builtin_elementwise_max(
                              __builtin_elementwise_max(__builtin_elementwise_sub_sat(e, vge), t),
                              zero));
      vf = __builtin_elementwise_max(__builtin_elementwise_sub_sat(vf, vge), t);
      vh = ld(hl + s * kLanes);                           // diagonal of segment s + 1
    }
    // F leaving each lane's last row enters the next lane's first row.  The
    // correction carries vf down the column: where it exceeds H it raises H
    // (and the next column's E); a raised H adds nothing below that vf - ge
    // does not (H - go <= vf - ge), so only vf moves on.  It stops once vf -
    // ge is at most H - go of the row it leaves, taken before the raise: the
    // F already entering the next row (in the column pass or an earlier
    // correction) is at least that, and so dominates vf from there down.
    vf = __builtin_elementwise_max(shift_up(vf), zero);
    for (int pass = 0; pass < kLanes; ++pass) {
      bool more = true;
      for (int s = 0; s < seg; ++s) {
        v16 h = ld(hs + s * kLanes);
        const v16 t_old = __builtin_elementwise_sub_sat(h, vgo);
        if (any_gt(vf, h)) {
          h = __builtin_elementwise_max(h, vf);
          vmax = __builtin_elementwise_max(vmax, h);
          st(hs + s * kLanes, h);
          st(ev + s * kLanes, __builtin_elementwise_max(ld(ev + s * kLanes),
                                                        __builtin_elementwise_sub_sat(h, vgo)));
        }
        vf = __builtin_elementwise_max(__builtin_elementwise_sub_sat(vf, vge), zero);
        if (!any_gt(vf, t_old)) { more = false; break; }
      }
      if (!more) break;
      vf = __builtin_elementwise_max(shift_up(vf), zero);
    }
    std::swap(hl, hs);
  }
  const int32_t best = __builtin_reduce_max(vmax);
  return best >= kSat ? -1 : best;
}

__attribute__((target("avx2"))) int32_t striped_avx2(const Profile& p, const uint8_t* seq, int n,
                                                     int32_t go, int32_t ge, Workspace* w) {
  return striped(p, seq, n, go, ge, w);
}

int32_t striped_generic(const Profile& p, const uint8_t* seq, int n, int32_t go, int32_t ge,
                        Workspace* w) {
  return striped(p, seq, n, go, ge, w);
}

// The recurrence in 32-bit scalar arithmetic (sequences whose 16-bit
// maximum saturated), E and F floored at 0 like the vector form.
int32_t scalar32(const Profile& p, const uint8_t* seq, int n, int32_t go, int32_t ge,
                 Workspace* w) {
  const int m = p.m;
  w->hrow.assign((size_t)n + 1, 0);
  w->frow.assign((size_t)n + 1, 0);
  int32_t* hr = w->hrow.data();
  int32_t* fr = w->frow.data();
  int32_t best = 0;
  for (int i = 0; i < m; ++i) {
    const int8_t* srow = p.rows.data() + (size_t)i * 24;
    int32_t diag = 0, left = 0, e = 0;
    for (int j = 1; j <= n; ++j) {
      const int32_t up = hr[j];
      int32_t h = diag + srow[seq[j - 1]];
      h = std::max(h, std::max(e, fr[j]));
      h = std::max(h, 0);
      best = std::max(best, h);
      diag = up;
      hr[j] = h;
      left = h;
      e = std::max(std::max(e - ge, left - go), 0);
      fr[j] = std::max(std::max(fr[j] - ge, h - go), 0);
    }
  }
  return best;
}

}  // namespace

bool has_avx2() {
  static const bool yes = __builtin_cpu_supports("avx2");
  return yes;
}

void build_profile(const uint8_t* query, int m, const int8_t* matrix, Profile* p) {
  p->m = m;
  p->seg = std::max(1, (m + kLanes - 1) / kLanes);
  p->v.assign((size_t)kCodes * p->seg * kLanes, kPadScore);
  for (int c = 0; c < kCodes; ++c)
    for (int s = 0; s < p->seg; ++s)
      for (int k = 0; k < kLanes; ++k) {
        const int i = k * p->seg + s;
        if (i < m && c != kPad && query[i] < 24)
          p->v[((size_t)c * p->seg + s) * kLanes + k] = matrix[query[i] * 24 + c];
      }
  p->rows.assign((size_t)m * 24, 0);
  for (int i = 0; i < m; ++i)
    for (int c = 0; c < 24; ++c)
      p->rows[(size_t)i * 24 + c] = query[i] < 24 ? matrix[query[i] * 24 + c] : kPadScore;
}

int32_t score(const Profile& p, const uint8_t* seq, int n, int32_t go, int32_t ge, Workspace* w) {
  if (p.m == 0 || n == 0) return 0;
  const size_t need = (size_t)p.seg * kLanes;
  if (w->h0.size() < need) {
    w->h0.resize(need);
    w->h1.resize(need);
    w->e.resize(need);
  }
  const int32_t s = has_avx2() ? striped_avx2(p, seq, n, go, ge, w)
                               : striped_generic(p, seq, n, go, ge, w);
  return s >= 0 ? s : scalar32(p, seq, n, go, ge, w);
}

}  // namespace cpu
}  // namespace swdb
