// Internal declarations shared by the host runtime and the kernel sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/swdb.h"

namespace swdb {

// One bin of SW_BIN_SEQS short sequences (layout documented in swdb.h).
struct BinDesc {
  int64_t res_off;   // dword offset of the bin in the interleaved store
  int64_t rb_off;    // offset of the bin's boundary-row buffer, in uint4 units
  int64_t len;       // padded length (columns), multiple of 4, >= SW_MIN_BIN_LEN
  int64_t slot0;     // index of the bin's first slot in slot_seq
};
static_assert(sizeof(BinDesc) == 32, "BinDesc must match the 4 x int64 host layout");

// Scoring matrix passed by value to the profile kernel.
struct Matrix {
  int8_t v[SW_ALPHA * SW_ALPHA];
};

// Inter-task profile: for each pair of query rows (2r, 2r+1), 26 dwords
// (codes 0..23, the pad code 24, one spare); dword (r, c) = score of row 2r
// against code c in bits 0..15, of row 2r+1 in bits 16..31.  13 dwords per
// query row.
constexpr int kProfPairDwords = 26;
constexpr int kProfRowDwords = 13;
// Score given to padding (pad code, and query rows past the end).  Any value
// <= 0 keeps padded cells from raising a maximum.
constexpr int kPadScore = -64;
// Intra-task profile (int8, [code][row]) has the 24 codes plus the pad code.
constexpr int kIntraCodes = 25;

struct InterArgs {
  const uint2* res2;          // interleaved store viewed as (lo, hi) dword pairs
  const BinDesc* bins;
  int32_t bin_begin;          // first bin of this launch
  int32_t n_strips;           // query strips of R rows
  const uint32_t* prof;       // [n_strips * R][13] dwords
  uint32_t go2, ge2;          // gap penalties replicated in both 16-bit halves
  uint4* rb;                  // boundary-row buffers of all bins
  const int32_t* slot_seq;
  int32_t* out;
  int32_t* flag_count;        // rescoring list: count, then sequence ids
  int32_t* flag_list;
  int32_t sat_limit;
};

struct IntraArgs {
  const uint8_t* res;         // contiguous residues, original order
  const int64_t* offs;
  const int32_t* items;       // sequence ids to score
  const int32_t* count_ptr;   // device item count (rescoring) or nullptr
  int32_t count;              // host item count when count_ptr == nullptr
  const int8_t* prof2;        // [25][m_pad2] int8
  int32_t m_pad2;             // multiple of 64*R for every R used with it
  int32_t n_pass;             // passes of 64*R rows covering the query
  int32_t go, ge;
  int2* scratch;              // per-workgroup boundary rows
  int64_t scratch_stride;     // int2 elements per workgroup
  int32_t* out;
};

// Kernel launchers (return hipSuccess or the launch error).
hipError_t launch_profile(const uint8_t* d_query, int m, const Matrix& mat, uint32_t* prof,
                          int m_pad, int8_t* prof2, int m_pad2, int32_t* flag_count,
                          hipStream_t s);
hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_inter(int R, int W, int n_bins, const InterArgs& a, hipStream_t s);
hipError_t launch_intra(int RR, int W2, int grid, const IntraArgs& a, hipStream_t s);

}  // namespace swdb
