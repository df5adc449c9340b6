// Host (CPU) scorer of the hybrid CPU + GPU search: the same local alignment
// scores as the GPU kernels, computed on host cores for the sequences the
// host takes from the shared work order (paper section 2.3: SW#db uses CPU
// and GPU at once with dynamic work distribution).
#pragma once
#include <stdint.h>

#include <vector>

namespace swdb {
namespace cpu {

// Query profile in Farrar's striped layout for 16 lanes of 16-bit integers:
// segment s, lane k holds query row k * seg + s, for 25 codes (the 24
// residue codes and the pad code); rows past the query's end hold the pad
// score.
struct Profile {
  int m = 0;
  int seg = 0;                 // segments: ceil(m / 16), at least 1
  std::vector<int16_t> v;      // [25][seg][16]
  std::vector<int8_t> rows;    // [m][24] substitution rows of the query (for rescoring)
};

void build_profile(const uint8_t* query, int m, const int8_t* matrix, Profile* p);

// Per-thread scratch of the striped kernel.
struct Workspace {
  std::vector<int16_t> h0, h1, e;   // seg x 16 each
  std::vector<int32_t> hrow, frow;  // rescoring rows
};

// Score of the query against one database sequence (codes < 24), exact:
// 16-bit striped SIMD, and 32-bit scalar rescoring when a 16-bit value
// saturates.  go, ge: 0 <= ge <= go.
int32_t score(const Profile& p, const uint8_t* seq, int n, int32_t go, int32_t ge, Workspace* w);

// True when the host CPU runs the 256-bit vector form.
bool has_avx2();

}  // namespace cpu
}  // namespace swdb
