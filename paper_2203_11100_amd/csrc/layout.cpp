// Host-only database layout: validation, length sort, bins, interleaving.
// Builds the position-major interleaved residue store in which neighbouring
// lanes read neighbouring dwords (the coalesced 2-D sequence array of paper
// section 3.2, figures "matrix_usm"/"matrix_read"), with sequences sorted by
// length so that the sequences sharing a wavefront have similar lengths.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/swdb.h"
#include "layout.h"

namespace swdb {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

int plan_layout(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
                int32_t long_threshold, Plan* plan) {
  if (n_seqs < 0) { set_error("n_seqs < 0"); return SW_EINVAL; }
  if (n_seqs > INT32_MAX) { set_error("more than 2^31-1 sequences"); return SW_ERANGE; }
  if (!offsets) { set_error("offsets is NULL"); return SW_EINVAL; }
  if (offsets[0] != 0) { set_error("offsets[0] must be 0"); return SW_EINVAL; }
  int32_t t_long = long_threshold <= 0 ? SW_DEFAULT_LONG_THRESHOLD : long_threshold;
  plan->long_threshold = t_long;
  plan->max_len = 0;
  for (int64_t i = 0; i < n_seqs; ++i) {
    int64_t l = offsets[i + 1] - offsets[i];
    if (l < 0) { set_error("offsets must be non-decreasing"); return SW_EINVAL; }
    if (l > SW_MAX_LEN) { set_error("sequence longer than 2^24-1 residues"); return SW_ERANGE; }
    if (l > plan->max_len) plan->max_len = (int32_t)l;
  }
  if (n_seqs > 0 && !residues && offsets[n_seqs] > 0 && plan->check_codes) {
    set_error("residues is NULL");
    return SW_EINVAL;
  }
  if (residues && plan->check_codes) {
    const int64_t N = offsets[n_seqs];
    for (int64_t p = 0; p < N; ++p)
      if (residues[p] >= SW_ALPHA) {
        set_error("residue code >= 24 at position " + std::to_string(p));
        return SW_EINVAL;
      }
  }
  // stable sort by decreasing length (ties keep the original order)
  plan->order.resize((size_t)n_seqs);
  std::iota(plan->order.begin(), plan->order.end(), 0);
  std::stable_sort(plan->order.begin(), plan->order.end(), [&](int32_t a, int32_t b) {
    return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
  });
  int64_t n_long = 0;
  while (n_long < n_seqs &&
         offsets[plan->order[n_long] + 1] - offsets[plan->order[n_long]] >= t_long)
    ++n_long;
  // the very long sequences (a prefix of the long list) stay out of the long
  // bins; with the 32-bit threshold t_vlong = 4 * t_long
  const int64_t t_vlong = 4 * (int64_t)t_long;
  int64_t n_vlong = 0;
  while (n_vlong < n_long &&
         offsets[plan->order[n_vlong] + 1] - offsets[plan->order[n_vlong]] >= t_vlong)
    ++n_vlong;
  plan->n_long = n_long;
  plan->n_vlong = n_vlong;
  plan->very_long_threshold = (int32_t)std::min<int64_t>(t_vlong, INT32_MAX);
  plan->max_long_len = n_long ? (int32_t)(offsets[plan->order[0] + 1] - offsets[plan->order[0]]) : 0;
  const int64_t n_short = n_seqs - n_long;
  plan->n_bins = (n_short + SW_BIN_SEQS - 1) / SW_BIN_SEQS;
  plan->n_long_bins = (n_long - n_vlong + SW_BIN_SEQS - 1) / SW_BIN_SEQS;
  const int64_t n_all = plan->n_bins + plan->n_long_bins;
  plan->bins.resize((size_t)n_all * 4);
  plan->bin_first.resize((size_t)n_all);
  plan->bin_count.resize((size_t)n_all);
  int64_t res_off = 0, rb_off = 0;
  plan->max_bin_len = 0;
  plan->max_short_len = 0;
  plan->max_all_bin_len = 0;
  for (int64_t b = 0; b < n_all; ++b) {
    // short bins cover order[n_long ..), long bins order[n_vlong .. n_long)
    const bool is_long = b >= plan->n_bins;
    const int64_t lb = is_long ? b - plan->n_bins : b;
    const int64_t first = (is_long ? n_vlong : n_long) + lb * SW_BIN_SEQS;
    const int64_t end_ = is_long ? n_long : n_seqs;
    plan->bin_first[(size_t)b] = first;
    plan->bin_count[(size_t)b] = (int32_t)std::min<int64_t>(SW_BIN_SEQS, end_ - first);
    // the first sequence of a bin is its longest
    const int32_t sid0 = plan->order[(size_t)first];
    const int64_t l = offsets[sid0 + 1] - offsets[sid0];
    if (!is_long && l > plan->max_short_len) plan->max_short_len = (int32_t)l;
    const int64_t len = std::max<int64_t>((l + 3) & ~int64_t(3), SW_MIN_BIN_LEN);
    int64_t* d = &plan->bins[(size_t)b * 4];
    d[0] = res_off;
    d[1] = rb_off;
    d[2] = len;
    d[3] = b * SW_BIN_SEQS;
    res_off += (len / 4) * SW_BIN_SEQS;
    rb_off += (len / 4) * 64 * 2;  // per 4 columns and lane: 2 x uint4 (H, F of 2 halves)
    if (!is_long && len > plan->max_bin_len) plan->max_bin_len = (int32_t)len;
    if (len > plan->max_all_bin_len) plan->max_all_bin_len = (int32_t)len;
  }
  plan->packed_dwords = res_off;
  plan->boundary_uint4 = rb_off;
  return SW_OK;
}

void fill_layout(const uint8_t* residues, const int64_t* offsets, const Plan& plan,
                 uint32_t* packed, int64_t* bin_desc, int32_t* slot_seq, int32_t* long_ids) {
  for (int64_t t = 0; t < plan.n_long; ++t) long_ids[t] = plan.order[(size_t)t];
  if (bin_desc) memcpy(bin_desc, plan.bins.data(), plan.bins.size() * sizeof(int64_t));
  const int64_t n_all = plan.n_bins + plan.n_long_bins;
  for (int64_t b = 0; b < n_all; ++b) {
    const int64_t* d = &plan.bins[(size_t)b * 4];
    const int64_t res_off = d[0], len = d[2];
    for (int k = 0; k < SW_BIN_SEQS; ++k) {
      const int64_t t = b * SW_BIN_SEQS + k;
      const int32_t sid = k < plan.bin_count[(size_t)b] ? plan.order[(size_t)(plan.bin_first[(size_t)b] + k)] : -1;
      slot_seq[t] = sid;
      const uint8_t* s = sid >= 0 ? residues + offsets[sid] : nullptr;
      const int64_t sl = sid >= 0 ? offsets[sid + 1] - offsets[sid] : 0;
      for (int64_t p = 0; p < len; p += 4) {
        uint32_t w = 0;
        for (int x = 0; x < 4; ++x) {
          const uint32_t c = (p + x < sl) ? s[p + x] : (uint32_t)SW_PAD_CODE;
          w |= (c << 3) << (8 * x);   // 8 x code: byte offset in a profile row pair
        }
        packed[res_off + (p / 4) * SW_BIN_SEQS + k] = w;
      }
    }
  }
}

}  // namespace swdb

extern "C" {

int sw_plan(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
            int32_t long_threshold, sw_plan_info* info) {
  if (!info) { swdb::set_error("info is NULL"); return SW_EINVAL; }
  swdb::Plan plan;
  plan.check_codes = residues != nullptr;
  int rc = swdb::plan_layout(residues, offsets, n_seqs, long_threshold, &plan);
  if (rc != SW_OK) return rc;
  info->n_bins = plan.n_bins;
  info->n_long_bins = plan.n_long_bins;
  info->n_long = plan.n_long;
  info->n_very_long = plan.n_vlong;
  info->very_long_threshold = plan.very_long_threshold;
  info->packed_dwords = plan.packed_dwords;
  info->boundary_bytes = plan.boundary_uint4 * 16;
  info->max_len = plan.max_len;
  info->max_bin_len = plan.max_bin_len;
  info->max_long_len = plan.max_long_len;
  info->long_threshold = plan.long_threshold;
  swdb::set_error("");
  return SW_OK;
}

int sw_pack(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
            int32_t long_threshold, uint32_t* packed, int64_t* bin_desc, int32_t* slot_seq,
            int32_t* long_ids) {
  swdb::Plan plan;
  plan.check_codes = true;
  int rc = swdb::plan_layout(residues, offsets, n_seqs, long_threshold, &plan);
  if (rc != SW_OK) return rc;
  if ((plan.packed_dwords && !packed) ||
      (plan.n_bins + plan.n_long_bins && (!bin_desc || !slot_seq)) ||
      (plan.n_long && !long_ids)) {
    swdb::set_error("an output array is NULL");
    return SW_EINVAL;
  }
  swdb::fill_layout(residues, offsets, plan, packed, bin_desc, slot_seq, long_ids);
  swdb::set_error("");
  return SW_OK;
}

const char* sw_last_error(void) { return swdb::get_error(); }

}  // extern "C"
