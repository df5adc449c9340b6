// Host runtime behind the C ABI in include/swdb.h: database upload, per-query
// profile construction, kernel dispatch over the inter-task bins and the
// intra-task long list, exact rescoring of saturated sequences, and timing.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "layout.h"

namespace swdb {
namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SW_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;   // elements
  hipError_t reserve(size_t n) {
    if (n <= cap && p) return hipSuccess;
    if (p) {
      // earlier kernels may still read the old buffer
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
      p = nullptr;
      cap = 0;
    }
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), n * sizeof(T));
    if (e == hipSuccess) cap = n;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

constexpr int kIntraGridLong = 1024;   // workgroups sweeping the long list
constexpr int kIntraGridRescore = 512; // workgroups sweeping the rescoring list

}  // namespace
}  // namespace swdb

struct sw_db {
  int device = 0;
  int64_t n_seqs = 0, n_res = 0;
  swdb::Plan plan;
  std::vector<int32_t> long_ids;
  int64_t long_residues = 0;

  // resident database
  swdb::DevBuf<uint32_t> packed;
  swdb::DevBuf<swdb::BinDesc> bins;
  swdb::DevBuf<int32_t> slot_seq;
  swdb::DevBuf<uint4> rb;          // inter-task boundary rows, all bins
  swdb::DevBuf<uint8_t> res;       // contiguous residues (original order)
  swdb::DevBuf<int64_t> offs;
  swdb::DevBuf<int32_t> d_long_ids;
  swdb::DevBuf<int2> rb_long;      // intra-task boundary rows, per workgroup
  swdb::DevBuf<int2> rb_resc;
  swdb::DevBuf<int32_t> flags;     // [0] count, [1..] rescoring list

  // per-query buffers, grown on demand
  swdb::DevBuf<uint32_t> prof;
  swdb::DevBuf<int8_t> prof2;
  swdb::DevBuf<uint8_t> q_stage;
  swdb::DevBuf<int32_t> out_stage;

  hipStream_t own_stream = nullptr;  // sync API
  hipStream_t aux_stream = nullptr;  // long-sequence kernel, overlapped
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // timing: (kind, start, end) event pairs recorded since the last
  // sw_get_stats; events are recycled through `ev_pool`
  struct Timed { int kind; hipEvent_t a, b; };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> ev_pool;

  // options
  bool timing = false;
  int32_t sat_limit = 32767;
  int32_t opt_rows = 0, opt_waves = 0, opt_intra_rows = 0, opt_intra_waves = 0;

  // bookkeeping since the last sw_get_stats
  sw_stats stats{};

  std::mutex mtx;
};

namespace swdb {
namespace {

void destroy(sw_db* db) {
  if (!db) return;
  DeviceGuard g(db->device);
  if (db->own_stream) (void)hipStreamSynchronize(db->own_stream);
  if (db->aux_stream) (void)hipStreamSynchronize(db->aux_stream);
  db->packed.release(); db->bins.release(); db->slot_seq.release(); db->rb.release();
  db->res.release(); db->offs.release(); db->d_long_ids.release(); db->rb_long.release();
  db->rb_resc.release(); db->flags.release(); db->prof.release(); db->prof2.release();
  db->q_stage.release(); db->out_stage.release();
  for (hipEvent_t* e : {&db->ev_fork, &db->ev_join})
    if (*e) (void)hipEventDestroy(*e);
  for (auto& t : db->timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  for (hipEvent_t e : db->ev_pool) (void)hipEventDestroy(e);
  if (db->own_stream) (void)hipStreamDestroy(db->own_stream);
  if (db->aux_stream) (void)hipStreamDestroy(db->aux_stream);
  delete db;
}

int validate_search(const sw_db* db, const void* query, int32_t m, const int8_t* matrix,
                    int32_t go, int32_t ge, const void* out) {
  if (!db) return fail(SW_EINVAL, "db is NULL");
  if (m < 0) return fail(SW_EINVAL, "query_len < 0");
  if (m > SW_MAX_LEN) return fail(SW_ERANGE, "query longer than 2^24-1 residues");
  if (m > 0 && !query) return fail(SW_EINVAL, "query is NULL");
  if (!matrix) return fail(SW_EINVAL, "matrix is NULL");
  if (db->n_seqs > 0 && !out) return fail(SW_EINVAL, "out_scores is NULL");
  if (ge < 0 || go < ge) return fail(SW_EINVAL, "gaps must satisfy 0 <= gap_extend <= gap_open");
  if (go > SW_MAX_GAP) return fail(SW_ERANGE, "gap_open > 2^30");
  return SW_OK;
}

int pick_rows(const sw_db* db, int m) {
  if (db->opt_rows) return db->opt_rows;
  const int pad32 = (m + 31) / 32 * 32, pad16 = (m + 15) / 16 * 16;
  return (pad32 - m) * 16 <= (pad16 - m) * 16 + m / 8 ? 32 : 16;  // R=32 unless it pads much more
}

int pick_waves(const sw_db* db, int n_strips) {
  if (db->opt_waves) return db->opt_waves;
  // more waves per bin shortens each bin's strip pipeline; measured best at 8
  // even when some waves idle in the last round
  (void)n_strips;
  return 8;
}

// Rows per lane (R) and waves (W2) of the intra-task kernel for a query of
// length m: the smallest estimated latency for one long sequence, where a
// pass of 64R rows costs about (10R + 10) VALU ops per step, waves beyond one
// per SIMD share it, and the passes run in rounds of W2.
void pick_intra(const sw_db* db, int m, int max_waves, int* R_out, int* W2_out) {
  double best = 1e300;
  int bR = 8, bW = 1;
  for (int R : {2, 4, 8}) {
    if (db->opt_intra_rows && R != db->opt_intra_rows) continue;
    const int passes = (m + 64 * R - 1) / (64 * R);
    for (int W2 : {1, 2, 4, 8}) {
      if (W2 > max_waves) continue;
      if (db->opt_intra_waves && max_waves > 2 && W2 != db->opt_intra_waves) continue;
      const int rounds = (passes + W2 - 1) / W2;
      const double share = W2 > 4 ? W2 / 4.0 : 1.0;
      const double est = rounds * (10.0 * R + 10.0) * share + 1e-3 * W2;
      if (est < best) { best = est; bR = R; bW = W2; }
    }
  }
  *R_out = bR;
  *W2_out = bW;
}

enum TimedKind { kTimeTotal = 0, kTimeInter = 1, kTimeIntra = 2, kTimeRescore = 3 };

hipEvent_t pool_event(sw_db* db) {
  if (!db->ev_pool.empty()) {
    hipEvent_t e = db->ev_pool.back();
    db->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start event of a timed region on stream s (no-op when timing is
// off); returns the index to close with time_end.
int time_begin(sw_db* db, int kind, hipStream_t s) {
  if (!db->timing) return -1;
  hipEvent_t a = pool_event(db), b = pool_event(db);
  if (!a || !b) return -1;
  if (hipEventRecord(a, s) != hipSuccess) return -1;
  db->timed.push_back({kind, a, b});
  return (int)db->timed.size() - 1;
}

void time_end(sw_db* db, int idx, hipStream_t s) {
  if (idx < 0) return;
  (void)hipEventRecord(db->timed[(size_t)idx].b, s);
}

// Enqueues one query's search on stream s.  All arguments validated.
int enqueue_search(sw_db* db, const uint8_t* d_query, int32_t m, const Matrix& mat, int32_t go,
                   int32_t ge, int32_t* d_out, hipStream_t s) {
  hipError_t e;
  if (db->n_seqs == 0) return SW_OK;
  if (m == 0) {
    e = launch_fill(d_out, db->n_seqs, 0, s);
    return e == hipSuccess ? SW_OK : hip_fail(e, "fill");
  }
  const int R = pick_rows(db, m);
  const int m_pad = (m + R - 1) / R * R;
  const int n_strips = m_pad / R;
  const int W = pick_waves(db, n_strips);
  int RR = 8, W2 = 1, RRr = 8, W2r = 1;
  pick_intra(db, m, 8, &RR, &W2);     // long sequences
  pick_intra(db, m, 2, &RRr, &W2r);   // rescoring (usually empty)
  // one intra-task profile serves both launches: pad to the larger pass
  const int rows2 = 64 * std::max(RR, RRr);
  const int m_pad2 = (m + rows2 - 1) / rows2 * rows2;

  if ((e = db->prof.reserve((size_t)m_pad * kProfRowDwords)) != hipSuccess)
    return fail(SW_ENOMEM, std::string("profile allocation: ") + hipGetErrorString(e));
  if ((e = db->prof2.reserve((size_t)kIntraCodes * m_pad2)) != hipSuccess)
    return fail(SW_ENOMEM, std::string("profile allocation: ") + hipGetErrorString(e));

  const int t_total = time_begin(db, kTimeTotal, s);
  if ((e = launch_profile(d_query, m, mat, db->prof.p, m_pad, db->prof2.p, m_pad2, db->flags.p,
                          s)) != hipSuccess)
    return hip_fail(e, "profile kernel");

  // long sequences: intra-task kernel on the auxiliary stream, overlapped
  // with the inter-task bins
  IntraArgs ia{};
  ia.res = db->res.p;
  ia.offs = db->offs.p;
  ia.prof2 = db->prof2.p;
  ia.m_pad2 = m_pad2;
  ia.go = go;
  ia.ge = ge;
  ia.out = d_out;
  const int64_t n_long = db->plan.n_long;
  if (n_long > 0) {
    if ((e = hipEventRecord(db->ev_fork, s)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipStreamWaitEvent(db->aux_stream, db->ev_fork, 0)) != hipSuccess)
      return hip_fail(e, "stream wait");
    IntraArgs la = ia;
    la.items = db->d_long_ids.p;
    la.count_ptr = nullptr;
    la.count = (int32_t)n_long;
    la.scratch = db->rb_long.p;
    la.scratch_stride = std::max<int64_t>(db->plan.max_long_len, 1);
    la.n_pass = (m + 64 * RR - 1) / (64 * RR);
    const int grid = (int)std::min<int64_t>(n_long, kIntraGridLong);
    const int tl = time_begin(db, kTimeIntra, db->aux_stream);
    if ((e = launch_intra(RR, W2, grid, la, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "intra-task kernel");
    time_end(db, tl, db->aux_stream);
    if ((e = hipEventRecord(db->ev_join, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "event");
  }

  // short sequences: inter-task kernel over all bins
  InterArgs a{};
  a.res2 = reinterpret_cast<const uint2*>(db->packed.p);
  a.bins = db->bins.p;
  a.bin_begin = 0;
  a.n_strips = n_strips;
  a.prof = db->prof.p;
  const uint32_t go16 = (uint32_t)std::min<int32_t>(go, 65535);
  const uint32_t ge16 = (uint32_t)std::min<int32_t>(ge, 65535);
  a.go2 = go16 | (go16 << 16);
  a.ge2 = ge16 | (ge16 << 16);
  a.rb = db->rb.p;
  a.slot_seq = db->slot_seq.p;
  a.out = d_out;
  a.flag_count = db->flags.p;
  a.flag_list = db->flags.p + 1;
  a.sat_limit = db->sat_limit;
  const int n_bins = (int)db->plan.n_bins;
  if (n_bins > 0) {
    const int ti = time_begin(db, kTimeInter, s);
    if ((e = launch_inter(R, W, n_bins, a, s)) != hipSuccess) return hip_fail(e, "inter-task kernel");
    time_end(db, ti, s);
    ++db->stats.n_inter_launches;
    // exact rescoring of sequences whose 16-bit score saturated
    IntraArgs ra = ia;
    ra.items = db->flags.p + 1;
    ra.count_ptr = db->flags.p;
    ra.count = 0;
    ra.scratch = db->rb_resc.p;
    ra.scratch_stride = std::max<int64_t>(db->plan.max_bin_len, 1);
    ra.n_pass = (m + 64 * RRr - 1) / (64 * RRr);
    const int tr = time_begin(db, kTimeRescore, s);
    if ((e = launch_intra(RRr, W2r, kIntraGridRescore, ra, s)) != hipSuccess)
      return hip_fail(e, "rescoring kernel");
    time_end(db, tr, s);
  }
  if (n_long > 0 && (e = hipStreamWaitEvent(s, db->ev_join, 0)) != hipSuccess)
    return hip_fail(e, "stream wait");
  time_end(db, t_total, s);

  db->stats.rows = R;
  db->stats.waves = W;
  const int64_t long_res = db->long_residues;
  db->stats.inter_cells += (int64_t)m * (db->n_res - long_res);
  db->stats.intra_cells += (int64_t)m * long_res;
  return SW_OK;
}

}  // namespace
}  // namespace swdb

extern "C" {

int sw_db_load_ex(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
                  int32_t long_threshold, sw_db** out_db) {
  using namespace swdb;
  if (!out_db) return fail(SW_EINVAL, "out_db is NULL");
  *out_db = nullptr;
  sw_db* db = new (std::nothrow) sw_db();
  if (!db) return fail(SW_ENOMEM, "host allocation failed");
  db->plan.check_codes = true;
  int rc = plan_layout(residues, offsets, n_seqs, long_threshold, &db->plan);
  if (rc != SW_OK) { delete db; return rc; }
  hipError_t e = hipGetDevice(&db->device);
  if (e != hipSuccess) { delete db; return hip_fail(e, "no HIP device"); }
  DeviceGuard g(db->device);
  db->n_seqs = n_seqs;
  db->n_res = offsets[n_seqs];
  const Plan& P = db->plan;
  db->long_ids.resize((size_t)P.n_long);
  for (int64_t t = 0; t < P.n_long; ++t) {
    db->long_ids[(size_t)t] = P.order[(size_t)t];
    db->long_residues += offsets[P.order[(size_t)t] + 1] - offsets[P.order[(size_t)t]];
  }
  // host staging of the interleaved store
  std::vector<uint32_t> h_packed;
  std::vector<int64_t> h_bins;
  std::vector<int32_t> h_slots, h_long;
  try {
    h_packed.resize((size_t)P.packed_dwords);
    h_bins.resize((size_t)P.n_bins * 4);
    h_slots.resize((size_t)P.n_bins * SW_BIN_SEQS);
    h_long.resize((size_t)P.n_long);
  } catch (...) {
    destroy(db);
    return fail(SW_ENOMEM, "host staging allocation failed");
  }
  fill_layout(residues, offsets, P, h_packed.data(), h_bins.data(), h_slots.data(), h_long.data());

  auto alloc_fail = [&](hipError_t err, const char* what) {
    destroy(db);
    return fail(SW_ENOMEM, std::string(what) + ": " + hipGetErrorString(err));
  };
  if ((e = db->packed.reserve((size_t)P.packed_dwords)) != hipSuccess) return alloc_fail(e, "packed");
  if ((e = db->bins.reserve((size_t)P.n_bins)) != hipSuccess) return alloc_fail(e, "bins");
  if ((e = db->slot_seq.reserve(h_slots.size())) != hipSuccess) return alloc_fail(e, "slots");
  if ((e = db->rb.reserve((size_t)P.boundary_uint4)) != hipSuccess) return alloc_fail(e, "boundary");
  if ((e = db->res.reserve((size_t)db->n_res)) != hipSuccess) return alloc_fail(e, "residues");
  if ((e = db->offs.reserve((size_t)n_seqs + 1)) != hipSuccess) return alloc_fail(e, "offsets");
  if ((e = db->d_long_ids.reserve((size_t)P.n_long)) != hipSuccess) return alloc_fail(e, "long ids");
  const int64_t long_grid = std::min<int64_t>(P.n_long, kIntraGridLong);
  if ((e = db->rb_long.reserve((size_t)std::max<int64_t>(long_grid, 1) *
                               std::max<int32_t>(P.max_long_len, 1))) != hipSuccess)
    return alloc_fail(e, "long scratch");
  if ((e = db->rb_resc.reserve((size_t)kIntraGridRescore * std::max<int32_t>(P.max_bin_len, 1))) !=
      hipSuccess)
    return alloc_fail(e, "rescore scratch");
  if ((e = db->flags.reserve((size_t)P.n_bins * SW_BIN_SEQS + 1)) != hipSuccess)
    return alloc_fail(e, "flags");

  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  if ((e = up(db->packed.p, h_packed.data(), h_packed.size() * 4)) != hipSuccess ||
      (e = up(db->bins.p, h_bins.data(), h_bins.size() * 8)) != hipSuccess ||
      (e = up(db->slot_seq.p, h_slots.data(), h_slots.size() * 4)) != hipSuccess ||
      (e = up(db->res.p, residues, (size_t)db->n_res)) != hipSuccess ||
      (e = up(db->offs.p, offsets, ((size_t)n_seqs + 1) * 8)) != hipSuccess ||
      (e = up(db->d_long_ids.p, h_long.data(), h_long.size() * 4)) != hipSuccess) {
    destroy(db);
    return hip_fail(e, "database upload");
  }
  if ((e = hipStreamCreateWithFlags(&db->own_stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&db->aux_stream, hipStreamNonBlocking)) != hipSuccess) {
    destroy(db);
    return hip_fail(e, "stream creation");
  }
  for (hipEvent_t* ev : {&db->ev_fork, &db->ev_join})
    if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) {
      destroy(db);
      return hip_fail(e, "event creation");
    }
  *out_db = db;
  set_error("");
  return SW_OK;
}

int sw_db_load(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs, sw_db** out_db) {
  return sw_db_load_ex(residues, offsets, n_seqs, 0, out_db);
}

void sw_db_free(sw_db* db) { swdb::destroy(db); }

int sw_db_info(const sw_db* db, int64_t* n_seqs, int64_t* n_residues, int32_t* max_len,
               int64_t* n_long) {
  if (!db) return swdb::fail(SW_EINVAL, "db is NULL");
  if (n_seqs) *n_seqs = db->n_seqs;
  if (n_residues) *n_residues = db->n_res;
  if (max_len) *max_len = db->plan.max_len;
  if (n_long) *n_long = db->plan.n_long;
  return SW_OK;
}

int sw_search_async(sw_db* db, const uint8_t* d_query, int32_t query_len, const int8_t* matrix,
                    int32_t gap_open, int32_t gap_extend, int32_t* d_out_scores,
                    void* hip_stream) {
  using namespace swdb;
  int rc = validate_search(db, d_query, query_len, matrix, gap_open, gap_extend, d_out_scores);
  if (rc != SW_OK) return rc;
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->device);
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = enqueue_search(db, d_query, query_len, mat, gap_open, gap_extend, d_out_scores,
                      reinterpret_cast<hipStream_t>(hip_stream));
  if (rc == SW_OK) set_error("");
  return rc;
}

int sw_search(sw_db* db, const uint8_t* query, int32_t query_len, const int8_t* matrix,
              int32_t gap_open, int32_t gap_extend, int32_t* out_scores) {
  using namespace swdb;
  int rc = validate_search(db, query, query_len, matrix, gap_open, gap_extend, out_scores);
  if (rc != SW_OK) return rc;
  for (int32_t i = 0; i < query_len; ++i)
    if (query[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24 at position " + std::to_string(i));
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->device);
  hipError_t e;
  if ((e = db->q_stage.reserve((size_t)std::max(query_len, 1))) != hipSuccess ||
      (e = db->out_stage.reserve((size_t)std::max<int64_t>(db->n_seqs, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("staging allocation: ") + hipGetErrorString(e));
  hipStream_t s = db->own_stream;
  if (query_len > 0 &&
      (e = hipMemcpyAsync(db->q_stage.p, query, (size_t)query_len, hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return hip_fail(e, "query upload");
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = enqueue_search(db, db->q_stage.p, query_len, mat, gap_open, gap_extend, db->out_stage.p, s);
  if (rc != SW_OK) {
    (void)hipStreamSynchronize(s);
    return rc;
  }
  if (db->n_seqs > 0 &&
      (e = hipMemcpyAsync(out_scores, db->out_stage.p, (size_t)db->n_seqs * 4, hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    return hip_fail(e, "score download");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
  set_error("");
  return SW_OK;
}

static int validate_batch(const sw_db* db, const void* queries, const int64_t* qoffs, int32_t nq,
                          const int8_t* matrix, int32_t go, int32_t ge, const void* out) {
  using namespace swdb;
  if (!db) return fail(SW_EINVAL, "db is NULL");
  if (nq < 0) return fail(SW_EINVAL, "n_queries < 0");
  if (nq > 0 && !qoffs) return fail(SW_EINVAL, "query_offsets is NULL");
  if (nq > 0 && qoffs[0] != 0) return fail(SW_EINVAL, "query_offsets[0] must be 0");
  for (int32_t q = 0; q < nq; ++q) {
    const int64_t m = qoffs[q + 1] - qoffs[q];
    if (m < 0) return fail(SW_EINVAL, "query_offsets must be non-decreasing");
    if (m > SW_MAX_LEN) return fail(SW_ERANGE, "query longer than 2^24-1 residues");
  }
  if (nq > 0 && qoffs[nq] > 0 && !queries) return fail(SW_EINVAL, "queries is NULL");
  if (!matrix) return fail(SW_EINVAL, "matrix is NULL");
  if (nq > 0 && db->n_seqs > 0 && !out) return fail(SW_EINVAL, "out_scores is NULL");
  if (ge < 0 || go < ge) return fail(SW_EINVAL, "gaps must satisfy 0 <= gap_extend <= gap_open");
  if (go > SW_MAX_GAP) return fail(SW_ERANGE, "gap_open > 2^30");
  return SW_OK;
}

int sw_search_batch_async(sw_db* db, const uint8_t* d_queries, const int64_t* query_offsets,
                          int32_t n_queries, const int8_t* matrix, int32_t gap_open,
                          int32_t gap_extend, int32_t* d_out_scores, void* hip_stream) {
  using namespace swdb;
  int rc = validate_batch(db, d_queries, query_offsets, n_queries, matrix, gap_open, gap_extend,
                          d_out_scores);
  if (rc != SW_OK) return rc;
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->device);
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  for (int32_t q = 0; q < n_queries; ++q) {
    const int32_t m = (int32_t)(query_offsets[q + 1] - query_offsets[q]);
    rc = enqueue_search(db, d_queries + query_offsets[q], m, mat, gap_open, gap_extend,
                        d_out_scores + (size_t)q * db->n_seqs, s);
    if (rc != SW_OK) return rc;
  }
  set_error("");
  return SW_OK;
}

int sw_search_batch(sw_db* db, const uint8_t* queries, const int64_t* query_offsets,
                    int32_t n_queries, const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                    int32_t* out_scores) {
  using namespace swdb;
  int rc = validate_batch(db, queries, query_offsets, n_queries, matrix, gap_open, gap_extend,
                          out_scores);
  if (rc != SW_OK) return rc;
  const int64_t total = n_queries > 0 ? query_offsets[n_queries] : 0;
  for (int64_t i = 0; i < total; ++i)
    if (queries[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24 at position " + std::to_string(i));
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->device);
  hipError_t e;
  hipStream_t s = db->own_stream;
  if ((e = db->q_stage.reserve((size_t)std::max<int64_t>(total, 1))) != hipSuccess ||
      (e = db->out_stage.reserve((size_t)std::max<int64_t>(db->n_seqs, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("staging allocation: ") + hipGetErrorString(e));
  if (total > 0 &&
      (e = hipMemcpyAsync(db->q_stage.p, queries, (size_t)total, hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return hip_fail(e, "query upload");
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  for (int32_t q = 0; q < n_queries; ++q) {
    const int32_t m = (int32_t)(query_offsets[q + 1] - query_offsets[q]);
    rc = enqueue_search(db, db->q_stage.p + query_offsets[q], m, mat, gap_open, gap_extend,
                        db->out_stage.p, s);
    if (rc != SW_OK) { (void)hipStreamSynchronize(s); return rc; }
    if (db->n_seqs > 0 &&
        (e = hipMemcpyAsync(out_scores + (size_t)q * db->n_seqs, db->out_stage.p,
                            (size_t)db->n_seqs * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(e, "score download");
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
  set_error("");
  return SW_OK;
}

int sw_set_option(sw_db* db, int32_t key, int64_t value) {
  using namespace swdb;
  if (!db) return fail(SW_EINVAL, "db is NULL");
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  switch (key) {
    case SW_OPT_TIMING:
      if (value != 0 && value != 1) return fail(SW_EINVAL, "timing must be 0 or 1");
      db->timing = value != 0;
      return SW_OK;
    case SW_OPT_SAT_LIMIT:
      if (value < 0 || value > 32767) return fail(SW_EINVAL, "saturation limit must be in 0..32767");
      db->sat_limit = (int32_t)value;
      return SW_OK;
    case SW_OPT_ROWS:
      if (value != 0 && value != 16 && value != 32) return fail(SW_EINVAL, "rows must be 0, 16 or 32");
      db->opt_rows = (int32_t)value;
      return SW_OK;
    case SW_OPT_WAVES:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
        return fail(SW_EINVAL, "waves must be 0, 1, 2, 4 or 8");
      db->opt_waves = (int32_t)value;
      return SW_OK;
    case SW_OPT_INTRA_ROWS:
      if (value != 0 && value != 2 && value != 4 && value != 8)
        return fail(SW_EINVAL, "intra rows must be 0, 2, 4 or 8");
      db->opt_intra_rows = (int32_t)value;
      return SW_OK;
    case SW_OPT_INTRA_WAVES:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
        return fail(SW_EINVAL, "intra waves must be 0, 1, 2, 4 or 8");
      db->opt_intra_waves = (int32_t)value;
      return SW_OK;
    default:
      return fail(SW_EINVAL, "unknown option " + std::to_string(key));
  }
}

int sw_get_stats(sw_db* db, sw_stats* out) {
  using namespace swdb;
  if (!db || !out) return fail(SW_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->device);
  sw_stats st = db->stats;
  hipError_t e;
  hipEvent_t first = nullptr, last = nullptr;
  for (auto& t : db->timed) {
    if ((e = hipEventSynchronize(t.b)) != hipSuccess) return hip_fail(e, "event sync");
    float ms = 0;
    if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) continue;
    if (t.kind == kTimeInter) st.ms_inter += ms;
    if (t.kind == kTimeIntra) st.ms_intra += ms;
    if (t.kind == kTimeRescore) st.ms_rescore += ms;
    if (t.kind == kTimeTotal) {
      if (!first) first = t.a;
      last = t.b;
    }
  }
  float ms = 0;
  if (first && hipEventElapsedTime(&ms, first, last) == hipSuccess) st.ms_total = ms;
  for (auto& t : db->timed) { db->ev_pool.push_back(t.a); db->ev_pool.push_back(t.b); }
  db->timed.clear();
  int32_t cnt = 0;
  if (db->own_stream) (void)hipStreamSynchronize(db->own_stream);
  if (db->flags.p && db->plan.n_bins > 0) {
    if ((e = hipMemcpy(&cnt, db->flags.p, 4, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "stats");
  }
  st.n_rescored = cnt;
  *out = st;
  db->stats = sw_stats{};
  return SW_OK;
}

}  // extern "C"
