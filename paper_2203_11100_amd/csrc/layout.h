// Host-side database layout (shared by the runtime and the exported
// sw_plan/sw_pack functions).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace swdb {

struct Plan {
  bool check_codes = true;
  int32_t long_threshold = 0;
  int32_t very_long_threshold = 0;
  int32_t max_len = 0, max_bin_len = 0, max_long_len = 0, max_short_len = 0;
  int32_t max_all_bin_len = 0;  // including the long bins
  int64_t n_long = 0, n_vlong = 0, n_bins = 0, n_long_bins = 0;
  int64_t packed_dwords = 0, boundary_uint4 = 0;
  std::vector<int32_t> order;   // sorted original indices, longest first
  // bins: n_bins short bins, then n_long_bins bins of the long sequences
  // below the very-long threshold; {res_off, rb_off, len, slot0} each
  std::vector<int64_t> bins;
  std::vector<int64_t> bin_first;   // index into `order` of each bin's first slot
  std::vector<int32_t> bin_count;   // sequences in each bin
};

int plan_layout(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
                int32_t long_threshold, Plan* plan);
void fill_layout(const uint8_t* residues, const int64_t* offsets, const Plan& plan,
                 uint32_t* packed, int64_t* bin_desc, int32_t* slot_seq, int32_t* long_ids);

void set_error(const std::string& msg);
const char* get_error();

}  // namespace swdb
