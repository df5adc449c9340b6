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

// Profile rows: 26 codes per query row (codes 0..23, the pad code 24, one
// spare), one dword per row and code.  Rows are stored in pairs, code-major
// within a pair: the dword of row 2r + t and code c sits at
// r * kProfPairDwords + 2 * c + t, so one 64-bit LDS read at byte offset
// 8 * c returns both rows of a pair (the residue bytes of the interleaved
// store hold 8 x code).
constexpr int kProfRowDwords = 26;
constexpr int kProfPairDwords = 2 * kProfRowDwords;
constexpr uint32_t kHalfOne = 0x3c00u;   // binary16 1.0
// Inter-task profile, strip-major for strips of R rows: strip s holds two
// tables of R rows in the row-pair layout, the low table with dwords
// (S(a_i, c), 1) and the high table with dwords (1, S(a_i, c)), binary16
// (2 * R * kProfRowDwords dwords per strip).  A lane whose two sequences
// have residues x and y reads (S(a_i, x), 1) from the low table and
// (1, S(a_i, y)) from the high one; their packed product is (S(a_i, x),
// S(a_i, y)), so one packed fused multiply-add forms H_diag + S for both
// sequences.
__host__ __device__ constexpr int prof_strip_dwords(int R) { return 2 * R * kProfRowDwords; }
// Score given to padding (pad code, and query rows past the end).  Any value
// <= 0 keeps padded cells from raising a maximum.
constexpr int kPadScore = -64;
// Intra-task profile (int8, [code][row]) has the 24 codes plus the pad code.
constexpr int kIntraCodes = 25;

// The packed inter-task kernels compute in IEEE binary16, which holds every
// integer of magnitude <= 2048 exactly.
constexpr int kHalfExact = 2048;

// binary16 bit pattern of an integer n with |n| <= kHalfExact (exact).
__host__ __device__ constexpr uint16_t half_bits(int n) {
  const unsigned a = n < 0 ? (unsigned)-n : (unsigned)n;
  if (a == 0) return 0;
  const int e = 31 - __builtin_clz(a);
  const unsigned mant = (e <= 10 ? a << (10 - e) : a >> (e - 10)) & 0x3ffu;
  return (uint16_t)((n < 0 ? 0x8000u : 0u) | ((unsigned)(e + 15) << 10) | mant);
}
static_assert(half_bits(1) == 0x3c00 && half_bits(-64) == 0xd400 && half_bits(2048) == 0x6800 &&
                  half_bits(11) == 0x4980 && half_bits(0) == 0,
              "binary16 encodings");

struct InterArgs {
  const uint2* res2;          // interleaved store viewed as (lo, hi) dword pairs
  const BinDesc* bins;
  int32_t bin_begin;          // first bin of this launch
  int32_t n_strips;           // query strips of R rows
  const uint32_t* prof;       // n_strips * prof_strip_dwords(R) dwords
  uint32_t go2, ge2;          // gap penalties (binary16, capped at 2048) in both halves
  uint4* rb;                  // boundary-row buffers: bin b's at rb + (rb_off(b) - rb_base)
  int64_t rb_base;            // rb_off of the bin whose buffer starts at rb (0: all bins)
  const int32_t* slot_seq;
  int32_t* out;
  int32_t* flag_count;        // rescoring list: count, then {sid, query}
  int2* flag_list;
  int32_t sat_limit;          // rescoring limit, at most the exact range (see effective_limit)
};

// Per-query parameters of the intra-task kernel.
struct QueryDesc {
  int64_t prof2_off;          // byte offset of the query's [25][m_pad2] int8 profile
  int64_t out_off;            // offset of the query's score row in `out`
  int32_t m_pad2;             // profile row length: a multiple of 64*R
  int32_t n_pass;             // passes of 64*R rows covering the query
  int64_t prof3_off;          // dword offset of its packed [25][m_pad2 / 2] profile (batches)
  int32_t n_pass3;            // passes of the packed long-pair kernel (its own R)
  int32_t pad_;
};

struct IntraArgs {
  const uint8_t* res;         // contiguous residues, original order
  const int64_t* offs;
  const int2* items;          // {sequence id, query index}
  const int32_t* count_ptr;   // device item count (rescoring) or nullptr
  int32_t count;              // host item count when count_ptr == nullptr
  const int8_t* prof2;        // intra-task profiles of all queries
  QueryDesc q0;               // the query when `queries` is nullptr
  const QueryDesc* queries;   // per-query parameters (batched), or nullptr
  int32_t go, ge;
  int2* scratch;              // per-workgroup boundary rows
  int64_t scratch_stride;     // int2 elements per workgroup
  int32_t* out;
  int4* ends;                 // non-null: {sid, score, query end, db end} per item
                              // (end coordinates, instead of scores to `out`)
  int32_t mode;               // SW_MODE_*: local (with or without ends), global,
                              // semi-global (single query q0)
  int32_t m;                  // query length (global and semi-global)
  const int2* seg_items;      // non-null (ends): items {index into items, segment}
  int32_t seg_cols;           // over column windows as in IntraPairArgs
  int32_t seg_overlap;
  uint8_t* dir;               // non-null (with ends): the traceback codes of every
                              // cell, item it's at dir + dir_off[it], column-major
                              // with dir_ld bytes (>= the query's padded rows) per
                              // column; see k_intra.hip
  const int64_t* dir_off;
  int64_t dir_ld;
};

// Global / semi-global inter-task kernel (k_modes.hip): one database
// sequence per lane, strips of R query rows, int32.
struct ModeArgs {
  const uint32_t* res;        // interleaved store (dwords)
  const BinDesc* bins;
  const int32_t* slot_seq;
  const int64_t* offs;
  int32_t n_halfbins;         // 2 x short bins: one wave per half bin
  int32_t n_strips;
  int32_t m;
  int32_t go, ge;
  const int32_t* prof;        // [n_strips][26][R] int32
  int2* rb;                   // boundary rows: 4 x res_off + j * 128 + slot
  int32_t* out;
};

// Packed intra-task kernel for the long list of a single search: the two
// binary16 halves of a lane hold two database sequences (a pair) against
// the query.
struct IntraPairArgs {
  const uint8_t* res;         // contiguous residues, original order
  const int64_t* offs;
  const int2* items;          // {sequence a, sequence b or -1}, a not shorter
  int32_t count;
  const uint32_t* prof3;      // binary16 [25][m_pad2 / 2] row-pair dwords
  int32_t m_pad2;             // profile rows: a multiple of 64*R
  int32_t n_pass;             // passes of 64*R rows covering the query
  uint32_t go2, ge2;          // gap penalties (binary16, capped at 2048) in both halves
  int32_t sat_limit;
  int2* scratch;              // per-workgroup boundary rows {H pair, F pair}
  int64_t scratch_stride;     // int2 elements per workgroup
  int32_t* out;
  int32_t* flag_count;        // rescoring list: count, then {sid, query}
  int2* flag_list;
  // column segments (short queries): with seg_items non-null, item x is
  // {pair, segment}; segment s of a pair covers columns [s*seg_cols,
  // (s+1)*seg_cols) of its longer sequence and is computed over the window
  // that starts seg_overlap columns earlier, with a zero left border; the
  // item's packed maximum goes to seg_best[x] instead of `out`
  const int2* seg_items;
  int32_t seg_cols, seg_overlap;
  uint32_t* seg_best;
  // batches: with batch_items non-null, item x is {pair index into items,
  // query}, and the query's packed profile, pass count and score row come
  // from queries[query] (prof3 then points at all queries' profiles)
  const int2* batch_items;
  const QueryDesc* queries;
};

// Batched inter-task kernel: the two 16-bit halves of a lane hold two
// queries (a pair) against one database sequence.  The pair's profile has
// the inter-task layout (rows in pairs, code-major within a pair) with the
// dword of row i and code c holding (S(a_i, c), S(b_i, c)).
constexpr int kBatchRowDwords = kProfRowDwords;

struct PairDesc {
  int64_t prof_off;           // dword offset of the pair's [rows / 2][26][2] profile
  int32_t n_strips;           // strips of R rows covering the longer query
  int32_t qa, qb;             // query indices (qb < 0: high half unused)
  int32_t pad_;
};

struct BatchArgs {
  const uint32_t* res;        // interleaved store (dwords)
  const BinDesc* bins;
  const int2* items;          // {pair, 2 * bin + half}, costliest first
  int32_t n_items;
  int32_t* counter;           // work-queue head, zero at launch
  const PairDesc* pairs;
  const uint32_t* prof;
  uint32_t go2, ge2;
  uint4* rb;                  // per-workgroup boundary rows
  int64_t rb_stride;          // uint4 per workgroup
  const int32_t* slot_seq;
  int32_t* out;               // [n_queries][n_seqs]
  int64_t n_seqs;
  int32_t* flag_count;        // rescoring list: count, then {sid, query}
  int2* flag_list;
  int32_t sat_limit;
};

// Device state of the top-k selection (k_hits.hip): the radix histogram,
// the key digits fixed so far, how many keys equal to the prefix are still
// needed, the pass's finished-workgroup ticket, the count of keys above the
// final threshold collected so far, and per-workgroup counts of keys equal
// to the threshold.
constexpr int kTopkMaxBlocks = 512;
struct TopkState {
  uint32_t hist[256];
  uint32_t prefix;
  int32_t need;
  uint32_t done;
  int32_t n_gt;
  int32_t blockcnt[kTopkMaxBlocks];
};
static_assert(sizeof(TopkState) % 8 == 0, "TopkState keeps the arrays after it 8-byte aligned");

// Kernel launchers (return hipSuccess or the launch error).
hipError_t launch_profile(const uint8_t* d_query, int m, const Matrix& mat, uint32_t* prof,
                          int m_pad, int R, int8_t* prof2, uint32_t* prof3, int m_pad2,
                          int32_t* flag_count, hipStream_t s);
hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_inter(int R, int W, int n_bins, const InterArgs& a, hipStream_t s);
hipError_t launch_intra(int RR, int W2, int grid, const IntraArgs& a, hipStream_t s);
// R in {2, 4, 8}, W2 in {1, 2, 4, 8}, not (8, 8) (LDS)
hipError_t launch_intra_pairs(int R, int W2, int grid, const IntraPairArgs& a, hipStream_t s);
// Scores of segmented pairs: pair p's maximum over seg_best[seg0[p] ..
// seg0[p+1]), written to out (or the rescoring list) per half.
hipError_t launch_long_combine(const int2* pairs, const int32_t* seg0, int32_t n_pairs,
                               const uint32_t* seg_best, int32_t sat_limit, int32_t* out,
                               int32_t* flag_count, int2* flag_list, hipStream_t s);
hipError_t launch_batch(int R, int W, int grid, const BatchArgs& a, hipStream_t s);
int batch_workgroups_per_cu(int R, int W);
hipError_t launch_mode_profile(const uint8_t* d_query, int m, const Matrix& mat, int R,
                               int n_strips, int32_t* prof, int8_t* prof2, int m_pad2,
                               hipStream_t s);
hipError_t launch_mode_empty_query(const int64_t* offs, int64_t n_seqs, int mode, int go, int ge,
                                   int32_t* out, hipStream_t s);
// R in {16, 32}; mode SW_MODE_GLOBAL or SW_MODE_SEMIGLOBAL
hipError_t launch_mode_inter(int R, int mode, const ModeArgs& a, hipStream_t s);
// Top-k of scores[0 .. n): items[0 .. k) = {sequence, 0}, best first
// (1 <= k <= min(n, SW_MAX_TOPK)); gt and ties hold k int32 each.
hipError_t launch_topk(const int32_t* scores, int64_t n, int32_t k, TopkState* st, int32_t* gt,
                       int32_t* ties, int2* items, hipStream_t s);
// hits[i] = {items[i].x, 0, -1, -1}: the hit list of an empty query.
hipError_t launch_empty_hits(const int2* items, int32_t k, int4* hits, hipStream_t s);
// Column-segment items of k hits (seg0: k + 1 ints, seg_items: cap entries)
// and the per-hit combination of their ends (k_hits.hip).
hipError_t launch_hit_segments(const int2* items, int32_t k, const int64_t* offs, int32_t C,
                               int32_t cap, int32_t* seg0, int2* seg_items, hipStream_t s);
hipError_t launch_hit_combine(const int2* items, int32_t k, const int32_t* seg0,
                              const int4* seg_ends, int4* hits, hipStream_t s);
// Pair profiles for `n_pairs` pairs and intra-task profiles for `n_queries`
// queries of a batch (see k_misc.hip for the layouts); prof3 (or nullptr)
// receives the queries' packed long-pair profiles.
hipError_t launch_batch_profiles(const uint8_t* d_queries, const int64_t* d_qoffs, int n_queries,
                                 const Matrix& mat, const PairDesc* d_pairs, int n_pairs, int R,
                                 int64_t max_work, uint32_t* prof, const QueryDesc* d_qdesc,
                                 int8_t* prof2, uint32_t* prof3, hipStream_t s);

}  // namespace swdb
