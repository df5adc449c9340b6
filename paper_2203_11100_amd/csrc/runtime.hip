// Host runtime behind the C ABI in include/swdb.h: database upload, per-query
// profile construction, kernel dispatch over the inter-task bins and the
// intra-task long list, exact rescoring of saturated sequences, and timing.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include <atomic>
#include <condition_variable>
#include <memory>
#include <thread>

#include "cpu_scorer.h"
#include "trace_walk.h"
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

// HIP keeps the last failing call's error until hipGetLastError reads it,
// and the launch checks read it: an error already handled here is consumed
// so that it cannot surface at the next launch.
int hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(SW_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Work that may still use a searcher's buffers: its own two streams, and
// the last piece of work it enqueued on a caller's stream, marked by an
// event the searcher owns (recorded at the end of every call that enqueues
// on a caller's stream).  The caller's stream handle itself is never kept:
// the caller may destroy it once the call returns.  A buffer is only
// replaced after this work drains.
struct StreamSet {
  hipStream_t own[2] = {nullptr, nullptr};
  hipEvent_t caller_done = nullptr;
  bool caller_pending = false;
  bool any = false;
  void sync() const {
    if (!any) {
      (void)hipDeviceSynchronize();
      return;
    }
    for (hipStream_t s : own)
      if (s) (void)hipStreamSynchronize(s);
    if (caller_pending) (void)hipEventSynchronize(caller_done);
  }
};

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;   // elements
  const StreamSet* users = nullptr;
  hipError_t reserve(size_t n) {
    if (n <= cap && p) return hipSuccess;
    if (p) {
      // earlier kernels may still read the old buffer
      if (users) users->sync();
      else (void)hipDeviceSynchronize();
      (void)hipFree(p);
      p = nullptr;
      cap = 0;
    }
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), n * sizeof(T));
    if (e == hipSuccess) {
      cap = n;
    } else {
      p = nullptr;
      (void)hipGetLastError();   // handled by the caller: not a later launch's error
    }
    return e;
  }
  void release() {
    if (p) {
      if (users) users->sync();
      (void)hipFree(p);
    }
    p = nullptr;
    cap = 0;
  }
};

constexpr int kIntraGridLong = 1024;   // workgroups sweeping the long list
constexpr int kIntraGridRescore = 512; // workgroups sweeping the rescoring list

}  // namespace
}  // namespace swdb

// A prepared batch: device descriptors and profiles for one set of query
// lengths, matrix, gaps and buffers, plus the captured launch graph.
struct BatchPlan {
  bool valid = false;
  std::vector<int64_t> qoffs;
  swdb::Matrix mat{};
  int32_t go = 0, ge = 0, sat_limit = 0;
  const uint8_t* d_queries = nullptr;
  int32_t* d_out = nullptr;
  int R = 0, W = 0, RR = 0, W2 = 0, W2r = 0, RRp = 0, W2p = 0;
  int n_pairs = 0;
  int64_t n_items = 0, n_long_items = 0, max_pair_work = 0, max_query_work = 0;
  int64_t inter_cells = 0, intra_cells = 0;
  int grid_b = 0, grid_long = 0;
  std::vector<int32_t> zero_queries;
  swdb::DevBuf<swdb::PairDesc> pairs;
  swdb::DevBuf<swdb::QueryDesc> qdesc;
  swdb::DevBuf<int2> items;
  // the very long sequences in pairs, and the (pair, query) items of the
  // packed long-pair kernel, costliest first
  swdb::DevBuf<int2> vpairs, long_items;
  swdb::DevBuf<int64_t> qoffs_d;
  swdb::DevBuf<uint32_t> prof;
  swdb::DevBuf<int8_t> prof2;
  swdb::DevBuf<uint32_t> prof3;     // the queries' packed long-pair profiles
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the searcher's scratch buffers the captured graph's kernels address
  // (long-sequence and rescoring rows, rescoring list, work counter, batched
  // boundary rows): a searcher call that grows one of them frees the old
  // block, so the graph is re-captured whenever one of these differs
  const void* captured[5] = {};

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  void release() {
    drop_graph();
    pairs.release(); qdesc.release(); items.release(); long_items.release();
    vpairs.release(); qoffs_d.release(); prof.release(); prof2.release(); prof3.release();
    valid = false;
  }
};

namespace swdb {

// The resident database, shared by every search context of a handle.
struct DbData {
  int device = 0;
  int n_cus = 256;
  int64_t n_seqs = 0, n_res = 0;
  Plan plan;
  std::vector<int32_t> long_ids;
  std::vector<int32_t> long_len;    // by sequence id (only long ones set)
  int64_t long_residues = 0;        // all of the long list
  int64_t vlong_residues = 0;       // its very long prefix
  DevBuf<uint32_t> packed;          // interleaved bins
  DevBuf<BinDesc> bins;
  DevBuf<int32_t> slot_seq;
  DevBuf<uint8_t> res;              // contiguous residues (original order)
  DevBuf<int64_t> offs;
  DevBuf<int2> d_long_items;        // {sid, 0} for the long list
  DevBuf<int2> d_long_pairs;        // {sid a, sid b or -1}: the long list in pairs,
  int64_t n_long_pairs = 0;         // then the short bins' sequences in pairs
  // the short bins as pairs of neighbouring sequences, bin by bin from the
  // longest (bin 0), after the long pairs: a long query hands its longest
  // bins to the long-pair kernel.  bin_pair_end[b] = pairs of bins 0..b,
  // bin_res_cum[b] = residues of bins 0..b-1
  std::vector<int64_t> bin_pair_end, bin_res_cum;
  // column segments of the long pairs for short queries: seg_cols columns
  // each, items {pair, segment} pair by pair, pair p's items from
  // d_pair_seg0[p]; any_split when some pair has more than one
  int32_t seg_cols = 0;
  int64_t n_seg_items = 0;
  bool any_split = false;
  DevBuf<int2> d_seg_items;
  DevBuf<int32_t> d_pair_seg0;
  // host copies for the hybrid search's CPU share: residues, offsets, bin
  // descriptors {res_off, rb_off, len, slot0} and slots
  std::vector<uint8_t> h_res;
  std::vector<int64_t> h_offs, h_bins;
  std::vector<int32_t> h_slots;
};

// Host threads kept for the hybrid search's CPU share: run(n, f) starts
// f(0) .. f(n-1) on the first n threads (started on first use), wait()
// returns when all of them are done.  Starting threads per call had cost
// tens of microseconds each, per query.
struct HostPool {
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::vector<std::thread> threads;
  std::function<void(int)> job;
  int64_t gen = 0;
  int active = 0, running = 0;
  bool stop = false;

  void loop(int id) {
    int64_t seen = 0;
    for (;;) {
      std::function<void(int)> f;
      int n = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || gen != seen; });
        if (stop) return;
        seen = gen;
        f = job;
        n = active;
      }
      if (id < n) f(id);
      std::lock_guard<std::mutex> lk(mu);
      if (--running == 0) done_cv.notify_all();
    }
  }
  // throws std::system_error if a thread cannot be started
  void run(int n, std::function<void(int)> f) {
    while ((int)threads.size() < n) {
      const int id = (int)threads.size();
      threads.emplace_back([this, id] { loop(id); });
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      job = std::move(f);
      active = n;
      running = (int)threads.size();
      ++gen;
    }
    cv.notify_all();
  }
  void wait() {
    std::unique_lock<std::mutex> lk(mu);
    done_cv.wait(lk, [&] { return running == 0; });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto& t : threads) t.join();
  }
};

// Everything one search mutates: scratch buffers, streams, events, the
// batch plan, options and counters.  One call at a time per searcher.
struct Searcher {
  std::unique_ptr<HostPool> hpool;  // the hybrid search's host threads
  DbData* d = nullptr;
  StreamSet users;                  // streams this searcher's work runs on
  DevBuf<uint4> rb;                 // inter-task boundary rows, all short bins
  DevBuf<int2> rb_long;             // intra-task boundary rows, per workgroup
  DevBuf<int2> rb_resc;
  DevBuf<int32_t> flags;            // [0] count, [2..] {sid, query} rescoring list
  DevBuf<uint32_t> seg_best;        // packed maximum of every long-pair segment item
  DevBuf<uint32_t> prof;            // per-query buffers, grown on demand
  DevBuf<int8_t> prof2;
  DevBuf<uint32_t> prof3;           // binary16 row pairs of the packed intra-task kernel
  DevBuf<uint8_t> q_stage;
  DevBuf<int32_t> out_stage;
  BatchPlan batch;
  DevBuf<uint4> rb_batch;           // per-workgroup boundary rows of the batched kernel
  DevBuf<int32_t> counter;          // work-queue head of the batched kernel
  DevBuf<int32_t> topk;             // top-k selection state, candidates, hit items
  DevBuf<int4> hits_stage;          // hit list of host-buffer top-k calls
  DevBuf<uint8_t> trace_dir;        // traceback codes of one group of sequences
  DevBuf<int2> trace_items;         // {sequence, 0} of the group
  DevBuf<int64_t> trace_off;        // each item's code offset
  DevBuf<int4> trace_ends;          // each item's {sequence, score, query end, db end}
  DevBuf<int32_t> mprof;            // int32 strip profile of global / semi-global searches
  DevBuf<int2> rb_mode;             // their boundary rows, 8 bytes per short-bin cell column
  hipStream_t own_stream = nullptr; // host-buffer calls and batch graphs
  hipStream_t aux_stream = nullptr; // long-sequence kernel, overlapped
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_caller = nullptr;   // end of the last work enqueued on a caller's stream
  hipEvent_t ev_chunk[2] = {nullptr, nullptr};   // hybrid search: GPU chunks in flight
  // hybrid search: running averages of the GPU's short-bin rate and one host
  // thread's rate, cells per second (seeded low for the host, so that a
  // first call gives it little)
  double hyb_gpu_rate = 3e12, hyb_cpu_rate = 2e8;
  int32_t hyb_share = 0;            // SW_OPT_HYBRID_SHARE: fixed host share, thousandths
  // timing: (kind, start, end) event pairs recorded since the last
  // sw_get_stats; events are recycled through `ev_pool`
  struct Timed { int kind; hipEvent_t a, b; };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> ev_pool;
  // options
  bool timing = false;
  bool use_graphs = true;
  int32_t sat_limit = 32767;
  int32_t opt_rows = 0, opt_waves = 0, opt_intra_rows = 0, opt_intra_waves = 0;
  int64_t opt_offload = -1;         // short bins for the long-pair kernel: -1 automatic
  // autotuned (rows, waves) per query-length bucket; 0 = not tuned
  int32_t tune_rows[SW_TUNE_BUCKETS] = {}, tune_waves[SW_TUNE_BUCKETS] = {};
  int32_t tune_brows[SW_TUNE_BUCKETS] = {}, tune_bwaves[SW_TUNE_BUCKETS] = {};
  // autotuned (rows per lane, waves) of the long-pair kernel; 0 = not tuned
  int32_t tune_irows[SW_TUNE_BUCKETS] = {}, tune_iwaves[SW_TUNE_BUCKETS] = {};
  sw_stats stats{};                 // since the last sw_get_stats
  std::mutex mtx;
};

}  // namespace swdb

struct sw_db {
  swdb::DbData data;
  swdb::Searcher main;
};

struct sw_ctx {
  sw_db* owner = nullptr;
  swdb::Searcher s;
};

namespace swdb {
namespace {

// Releases a searcher's scratch, streams and events (not the database).
void release_searcher(Searcher* db) {
  if (db->own_stream) (void)hipStreamSynchronize(db->own_stream);
  if (db->aux_stream) (void)hipStreamSynchronize(db->aux_stream);
  db->rb.release(); db->rb_long.release(); db->rb_resc.release(); db->flags.release();
  db->seg_best.release();
  db->prof.release(); db->prof2.release(); db->prof3.release(); db->q_stage.release();
  db->out_stage.release();
  db->batch.release(); db->rb_batch.release(); db->counter.release();
  db->topk.release(); db->hits_stage.release(); db->mprof.release(); db->rb_mode.release();
  db->trace_dir.release(); db->trace_items.release(); db->trace_off.release();
  db->trace_ends.release();
  if (db->users.caller_pending) (void)hipEventSynchronize(db->ev_caller);
  db->users.caller_pending = false;
  for (hipEvent_t* e : {&db->ev_fork, &db->ev_join, &db->ev_in, &db->ev_out, &db->ev_caller,
                        &db->ev_chunk[0], &db->ev_chunk[1]}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  for (auto& t : db->timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  db->timed.clear();
  for (hipEvent_t e : db->ev_pool) (void)hipEventDestroy(e);
  db->ev_pool.clear();
  if (db->own_stream) (void)hipStreamDestroy(db->own_stream);
  if (db->aux_stream) (void)hipStreamDestroy(db->aux_stream);
  db->own_stream = db->aux_stream = nullptr;
  db->hpool.reset();
}

void destroy_db(sw_db* h) {
  if (!h) return;
  DeviceGuard g(h->data.device);
  release_searcher(&h->main);
  DbData& d = h->data;
  d.packed.release(); d.bins.release(); d.slot_seq.release(); d.res.release(); d.offs.release();
  d.d_long_items.release();
  d.d_long_pairs.release();
  d.d_seg_items.release();
  d.d_pair_seg0.release();
  delete h;
}

// Makes every buffer of a searcher wait for its streams before reallocation.
void bind_buffers(Searcher* S) {
  const StreamSet* u = &S->users;
  S->rb.users = S->rb_long.users = S->rb_resc.users = S->seg_best.users = u;
  S->prof.users = u; S->prof2.users = u; S->prof3.users = u; S->q_stage.users = u;
  S->out_stage.users = u;
  S->rb_batch.users = S->counter.users = S->flags.users = u;
  S->topk.users = S->hits_stage.users = u;
  S->trace_dir.users = S->trace_items.users = S->trace_off.users = S->trace_ends.users = u;
  S->mprof.users = S->rb_mode.users = u;
  BatchPlan& B = S->batch;
  B.pairs.users = u; B.qdesc.users = u; B.items.users = u; B.long_items.users = u;
  B.vpairs.users = u; B.qoffs_d.users = u; B.prof.users = u; B.prof2.users = u;
  B.prof3.users = u;
}

// Per-workgroup boundary-row length of the rescoring launch: any sequence of
// a bin or of the long list may be flagged.
int64_t rescore_stride(const Plan& P) {
  return std::max<int64_t>({(int64_t)P.max_all_bin_len, (int64_t)P.max_long_len, 1});
}

// Allocates a searcher's fixed scratch, streams and events for database d.
int init_searcher(Searcher* S, DbData* d) {
  S->d = d;
  bind_buffers(S);
  const Plan& P = d->plan;
  hipError_t e;
  if ((e = S->rb.reserve((size_t)P.boundary_uint4)) != hipSuccess ||
      (e = S->rb_resc.reserve((size_t)kIntraGridRescore * (size_t)rescore_stride(P))) !=
          hipSuccess ||
      (e = S->flags.reserve(
           (size_t)(2 + 2 * std::max<int64_t>(P.n_bins * SW_BIN_SEQS + P.n_long, 1)))) !=
          hipSuccess ||
      (e = S->seg_best.reserve((size_t)std::max<int64_t>(d->n_seg_items, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("search scratch: ") + hipGetErrorString(e));
  // the inter-task kernel's first strip reads zeros from the boundary rows;
  // every search leaves them zeroed again
  if ((e = hipMemset(S->rb.p, 0, (size_t)std::max<int64_t>(P.boundary_uint4, 1) * sizeof(uint4))) !=
      hipSuccess)
    return hip_fail(e, "boundary-row clear");
  if ((e = hipStreamCreateWithFlags(&S->own_stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&S->aux_stream, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "stream creation");
  S->users.own[0] = S->own_stream;
  S->users.own[1] = S->aux_stream;
  S->users.any = true;
  for (hipEvent_t* ev : {&S->ev_fork, &S->ev_join, &S->ev_in, &S->ev_out, &S->ev_caller,
                         &S->ev_chunk[0], &S->ev_chunk[1]})
    if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "event creation");
  S->users.caller_done = S->ev_caller;
  return SW_OK;
}

// Marks the end of the work a call enqueued on the caller's stream s, so
// later buffer replacements wait for it (without keeping s itself).
void mark_caller_work(Searcher* S, hipStream_t s) {
  if (hipEventRecord(S->ev_caller, s) == hipSuccess) S->users.caller_pending = true;
}

int validate_search(const Searcher* db, const void* query, int32_t m, const int8_t* matrix,
                    int32_t go, int32_t ge, const void* out) {
  if (!db) return fail(SW_EINVAL, "db is NULL");
  if (m < 0) return fail(SW_EINVAL, "query_len < 0");
  if (m > SW_MAX_LEN) return fail(SW_ERANGE, "query longer than 2^24-1 residues");
  if (m > 0 && !query) return fail(SW_EINVAL, "query is NULL");
  if (!matrix) return fail(SW_EINVAL, "matrix is NULL");
  if (db->d->n_seqs > 0 && !out) return fail(SW_EINVAL, "out_scores is NULL");
  if (ge < 0 || go < ge) return fail(SW_EINVAL, "gaps must satisfy 0 <= gap_extend <= gap_open");
  if (go > SW_MAX_GAP) return fail(SW_ERANGE, "gap_open > 2^30");
  return SW_OK;
}

int tune_bucket(int m) {
  static const int upper[SW_TUNE_BUCKETS - 1] = {256, 768, 2048};
  int b = 0;
  while (b < SW_TUNE_BUCKETS - 1 && m >= upper[b]) ++b;
  return b;
}

// Default schedule of the inter-task kernels: 16-row strips and 12 waves per
// bin (three waves per SIMD at 136 VGPRs; measured faster than 32 x 8 for
// every query length of the plain workload and for the batched one).
constexpr int kDefaultRows = 16, kDefaultWaves = 12;

// The fitted schedules of the single-query inter-task kernel: strip height
// R and waves W with a relative efficiency per strip slot, the median over
// the plain workload's queries of 700+ rows of GCUPS x padded rows / rows
// (scaled to 0.868 for 14 x 16): 12 waves (3 per SIMD) with 12..20 rows, 16
// waves (4 per SIMD, <= 128 VGPRs) with 12 or 14 rows.
struct Sched {
  int R, W;
  double eff;
};
constexpr Sched kScheds[] = {{20, 12, 0.835}, {18, 12, 0.821}, {16, 12, 0.838}, {14, 12, 0.810},
                             {12, 12, 0.814}, {14, 16, 0.868}, {12, 16, 0.863}};

// The batched kernel's fitted schedules, with relative efficiencies from the
// batched workload (220 queries, every form forced): GCUPS x padded rows /
// rows over its pairs, divided by 10,000.
constexpr Sched kBatchScheds[] = {{20, 12, 0.855}, {18, 12, 0.848}, {16, 12, 0.833},
                                  {14, 12, 0.845}, {12, 12, 0.834}, {14, 16, 0.843},
                                  {12, 16, 0.861}};

// A bin of C chunks takes ceil(S / W) rounds of its S = ceil(m / R) strips,
// each round C supersteps of W waves' chunks, so its time is proportional
// to ceil(S / W) * W * R / eff.  Picks the schedule minimising that among
// those with the given rows / waves (0: any); false if none matches.
bool fit_schedule(int m, int rows, int waves, int* R_out, int* W_out) {
  double best = 1e300;
  for (const Sched& c : kScheds) {
    if ((rows && c.R != rows) || (waves && c.W != waves)) continue;
    const int64_t rounds = ((m + c.R - 1) / c.R + c.W - 1) / c.W;
    const double cost = (double)rounds * c.W * c.R / c.eff;
    if (cost < best) { best = cost; *R_out = c.R; *W_out = c.W; }
  }
  return best < 1e300;
}

// Schedule of a single search: both options, else the autotuned entry of
// the query's bucket, else the fitted schedule (within a set option).
void pick_schedule(const Searcher* db, int m, int* R_out, int* W_out) {
  int R = db->opt_rows, W = db->opt_waves;
  const int b = tune_bucket(m);
  if (!(R && W)) {
    if (!R && !W && db->tune_waves[b]) {
      R = db->tune_rows[b];
      W = db->tune_waves[b];
    } else if (!fit_schedule(m, R, W, &R, &W)) {
      if (!R) R = kDefaultRows;
      if (!W) W = (R == 32) ? 8 : kDefaultWaves;
    }
  }
  if (W == 12 && R == 32) W = 8;                                 // no 12-wave form of 32 rows
  if (W == 16 && R != 12 && R != 14) fit_schedule(m, 0, 16, &R, &W);  // 16 waves: 12, 14
  if (W != 12 && W != 16 && R != 16 && R != 32) R = 16;          // 12..20 rows: 12 or 16 waves
  *R_out = R;
  *W_out = W;
}

// Rows per lane (R) and waves (W2) of the intra-task kernel for a query of
// length m: the smallest estimated latency for one long sequence, where a
// pass of 64R rows costs about (10R + 10) VALU ops per step in int32 and
// (8R + 24) in the packed binary16 kernel, waves beyond one per SIMD share
// it, and the passes run in rounds of W2.  The packed kernel has no (8, 8)
// (its LDS profile would exceed 160 KB).
void pick_intra(const Searcher* db, int m, int max_waves, int* R_out, int* W2_out,
                bool packed = false) {
  if (packed && !db->opt_intra_rows && !db->opt_intra_waves) {
    const int b = tune_bucket(m);
    if (db->tune_iwaves[b]) {     // the autotuned entry of the query's bucket
      *R_out = db->tune_irows[b];
      *W2_out = db->tune_iwaves[b];
      return;
    }
  }
  double best = 1e300;
  int bR = 8, bW = 1;
  for (int R : {2, 4, 8}) {
    if (db->opt_intra_rows && R != db->opt_intra_rows) continue;
    const int passes = (m + 64 * R - 1) / (64 * R);
    for (int W2 : {1, 2, 4, 8}) {
      if (W2 > max_waves) continue;
      if (packed && R == 8 && W2 == 8) continue;
      if (db->opt_intra_waves && max_waves > 2 && W2 != db->opt_intra_waves) continue;
      const int rounds = (passes + W2 - 1) / W2;
      const double share = W2 > 4 ? W2 / 4.0 : 1.0;
      const double step = packed ? 8.0 * R + 24.0 : 10.0 * R + 10.0;
      const double est = rounds * step * share + 1e-3 * W2;
      if (est < best) { best = est; bR = R; bW = W2; }
    }
  }
  if (best == 1e300 && packed) {   // only (8, 8) was allowed by the options
    bR = 8;
    bW = 4;
  }
  *R_out = bR;
  *W2_out = bW;
}

enum TimedKind { kTimeTotal = 0, kTimeInter = 1, kTimeIntra = 2, kTimeRescore = 3 };

hipEvent_t pool_event(Searcher* db) {
  if (!db->ev_pool.empty()) {
    hipEvent_t e = db->ev_pool.back();
    db->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();   // timing is skipped; not a later launch's error
    return nullptr;
  }
  return e;
}

// Records the start event of a timed region on stream s (no-op when timing is
// off); returns the index to close with time_end.
int time_begin(Searcher* db, int kind, hipStream_t s) {
  if (!db->timing) return -1;
  hipEvent_t a = pool_event(db), b = pool_event(db);
  if (!a || !b) return -1;
  if (hipEventRecord(a, s) != hipSuccess) return -1;
  db->timed.push_back({kind, a, b});
  return (int)db->timed.size() - 1;
}

void time_end(Searcher* db, int idx, hipStream_t s) {
  if (idx < 0) return;
  (void)hipEventRecord(db->timed[(size_t)idx].b, s);
}

// The rescoring list: flags[0] is the count, {sid, query} pairs start at
// flags + 2 (8-byte aligned).
int2* flag_list(Searcher* db) { return reinterpret_cast<int2*>(db->flags.p + 2); }

hipError_t reserve_flags(Searcher* db, int64_t entries) {
  return db->flags.reserve((size_t)(2 + 2 * std::max<int64_t>(entries, 1)));
}

hipError_t reserve_long_scratch(Searcher* db, int grid) {
  return db->rb_long.reserve((size_t)std::max(grid, 1) *
                             (size_t)std::max<int32_t>(db->d->plan.max_long_len, 1));
}

// Enqueues one query's search on stream s.  All arguments validated.
// Gap penalty for the half-precision kernels, in both halves: penalties
// above the exact range act like 2048 there (packed16.h).
uint32_t half_pair(int32_t g) {
  const uint32_t h = half_bits(std::min<int32_t>(g, kHalfExact));
  return h | (h << 16);
}

// Rescoring limit of the half-precision kernels: the requested limit, at
// most 2048, below which every value is computed exactly (packed16.h).
int32_t effective_limit(int32_t requested) {
  return std::max<int32_t>(0, std::min<int32_t>(requested, kHalfExact));
}

// Row length of a query's intra-task profiles: a whole number of the
// largest pass (64 lanes x 8 rows), so every (R, W2) can read them.
int intra_rows_pad(int m) { return (m + 511) / 512 * 512; }

// Boundary-row length one workgroup of the long-pair kernel needs for a
// column segment: a window is at most a segment plus an overlap no longer
// than a segment.
int64_t seg_stride(const DbData& d) {
  return std::max<int64_t>(1, std::min<int64_t>(d.plan.max_long_len, 2 * (int64_t)d.seg_cols));
}

// Columns a segment's window reaches back for a query of length m, or -1
// when the long pairs are not cut into segments for it.  A local alignment
// of positive score pairs r <= m residues of each sequence, gaining at most
// r * maxS, and every database column it skips costs at least gap_extend
// (a gap of k costs open + (k-1) extend >= k extend), so it skips fewer
// than r * maxS / extend columns and spans fewer than m + m * maxS / extend.
// A window starting that far before its segment therefore holds every
// positive-score alignment that ends in the segment, and the recurrence
// started there with a zero border gives exactly the true H in the
// segment's columns (lower bounds elsewhere).  Used when this reach is at
// most one segment (short queries) and extend > 0.
int64_t window_reach(int m, const Matrix& mat, int32_t ge) {
  int max_s = 0;
  for (int x = 0; x < SW_ALPHA * SW_ALPHA; ++x) max_s = std::max<int>(max_s, mat.v[x]);
  return (int64_t)m + ((int64_t)m * max_s + ge - 1) / ge;
}

int32_t seg_overlap(const DbData& d, int m, const Matrix& mat, int32_t ge) {
  if (!d.any_split || ge <= 0) return -1;
  const int64_t reach = window_reach(m, mat, ge);
  return reach <= d.seg_cols ? (int32_t)reach : -1;
}

// The same reach for the end pass over top-k hits, whose boundary rows hold
// a whole sequence: a window may then reach back more than one segment (it
// starts at column 0 at the latest), and cutting pays whenever a window is
// shorter than the longest sequence.  -1: whole sequences.
int32_t hit_overlap(const DbData& d, int m, const Matrix& mat, int32_t ge) {
  if (ge <= 0) return -1;
  const int64_t reach = window_reach(m, mat, ge);
  return (int64_t)d.plan.max_len > (int64_t)d.seg_cols + reach ? (int32_t)reach : -1;
}

// Schedule of one single-query search: inter-task strips (R rows, W waves),
// the packed long-sequence kernel (RR, W2), the rescoring kernel (RRr, W2r)
// and the intra-task profiles' row length.
struct SearchShape {
  int R, W, m_pad, n_strips, RR, W2, RRr, W2r, m_pad2;
  int64_t off_bins;   // the longest short bins handed to the long-pair kernel
};

// Rates of the search kernels on a 256-CU MI355X (cells per second),
// measured on the benchmark workloads: the inter-task kernel over the
// device, the long-pair kernel over the device, and one inter-task
// workgroup (one bin) alone on its CU.
constexpr double kInterRate = 7.0e12;
constexpr double kPairRate = 4.5e12;
constexpr double kBinRate = 3.0e10;

// How many of the longest short bins a query of length m hands to the
// long-pair kernel (RR query rows per lane).  A bin is 128 sequences on one
// workgroup, so it takes about m * len * 128 / kBinRate seconds however many
// CUs are free, while the search's whole work takes about inter cells /
// kInterRate + long-pair cells / kPairRate on the device (the pair rate
// scaled by the query rows' share of the passes' rows).  For a long query
// against few short sequences the longest bin outlasts that (the critical
// path of the inter-task kernel); in the long-pair kernel its sequences go
// two per workgroup and spread over the CUs.  When the longest bin would
// outlast the whole work, bins are handed over, longest first, until the
// longest remaining one ends within kOffloadMargin of it (the bin's own rate
// drops with the device's clock under full load, and the pair kernel takes
// the handed-over work beside its own).  Measured on the long-sequence mix,
// 6..16 bins hand over give the same time within 1 % (7 chosen), 8 % below
// none; on the plain workload, whose longest bin ends within the search's
// work, handing any over only adds time (2 bins +0.4 %, 40 bins +7 %).
constexpr double kOffloadMargin = 0.7;
int64_t pick_offload(const Searcher* db, int m, int RR) {
  const DbData& D = *db->d;
  const int64_t nb = D.plan.n_bins;
  if (db->opt_offload >= 0) return std::min<int64_t>(db->opt_offload, nb);
  if (nb == 0 || m <= 0 || RR <= 0 || D.bin_res_cum.size() != (size_t)nb + 1) return 0;
  const double cus = std::max(D.n_cus, 1) / 256.0;
  const int64_t pass_rows = 64 * (int64_t)RR;
  const double row_share = (double)m / (double)((m + pass_rows - 1) / pass_rows * pass_rows);
  const double inter_rate = kInterRate * cus, pair_rate = kPairRate * cus * row_share;
  double inter = (double)m * (double)(D.n_res - D.long_residues);
  double pair = (double)m * (double)D.long_residues;
  int64_t k = 0;
  while (k < nb) {
    const double t_bin = (double)m * (double)D.plan.bins[(size_t)k * 4 + 2] * SW_BIN_SEQS / kBinRate;
    if (t_bin <= (k > 0 ? kOffloadMargin : 1.0) * (inter / inter_rate + pair / pair_rate)) break;
    const double moved = (double)m * (double)(D.bin_res_cum[(size_t)k + 1] - D.bin_res_cum[(size_t)k]);
    inter -= moved;
    pair += moved;
    ++k;
  }
  return k;
}

// Boundary-row length one workgroup of the long-pair kernel needs for whole
// sequences: the longest long sequence, or the longest short one when short
// bins are handed over.
int64_t pair_stride(const DbData& d) {
  return std::max<int64_t>({(int64_t)d.plan.max_long_len, (int64_t)d.plan.max_short_len, 1});
}

SearchShape search_shape(const Searcher* db, int m) {
  SearchShape sh{};
  sh.R = kDefaultRows;
  sh.W = kDefaultWaves;
  pick_schedule(db, m, &sh.R, &sh.W);
  sh.m_pad = (m + sh.R - 1) / sh.R * sh.R;
  sh.n_strips = sh.m_pad / sh.R;
  sh.RR = 8; sh.W2 = 1; sh.RRr = 8; sh.W2r = 1;
  pick_intra(db, m, 8, &sh.RR, &sh.W2, true);   // long sequences, in pairs (binary16)
  // exact rescoring (usually a few sequences, each the only one on its CU,
  // so the latency of one sequence is what counts)
  pick_intra(db, m, 8, &sh.RRr, &sh.W2r);
  // the intra-task profiles serve every intra-task launch of the query (long
  // list, rescoring, hit ends): pad to the largest pass, 64 x 8 rows
  sh.m_pad2 = intra_rows_pad(m);
  sh.off_bins = pick_offload(db, m, sh.RR);
  return sh;
}

// Device scratch of one single-query search.
struct SearchScratch {
  uint4* rb = nullptr;        // boundary rows of every short bin, zero on entry
  int32_t* flags = nullptr;   // rescoring list: [0] count, {sid, query} pairs from +2
  uint32_t* prof = nullptr;   // inter-task strip profile
  int8_t* prof2 = nullptr;    // intra-task int8 profile
  uint32_t* prof3 = nullptr;  // packed intra-task profile (long list present)
  int2* rb_long = nullptr;    // per-workgroup rows of the long-sequence kernel
  int grid_long = 0;          // its workgroups over whole pairs
  int grid_seg = 0;           // and over column segments (rows of seg_stride)
  uint32_t* seg_best = nullptr;   // segment maxima (long list present)
  int2* rb_resc = nullptr;    // per-workgroup rows of the rescoring kernel
  int grid_resc = 0;
};

// Element counts of the scratch pieces above for a query of this shape.
struct ScratchSizes {
  size_t rb, flags, prof, prof2, prof3, rb_long, rb_resc;   // elements of each type
};

ScratchSizes scratch_sizes(const Searcher* db, const SearchShape& sh, int grid_long,
                           int grid_resc) {
  const Plan& P = db->d->plan;
  ScratchSizes z{};
  z.rb = (size_t)std::max<int64_t>(P.boundary_uint4, 1);
  z.flags = (size_t)(2 + 2 * std::max<int64_t>(P.n_bins * SW_BIN_SEQS + P.n_long, 1));
  z.prof = (size_t)sh.n_strips * prof_strip_dwords(sh.R);
  z.prof2 = (size_t)kIntraCodes * sh.m_pad2;
  z.prof3 = P.n_long > 0 ? (size_t)kIntraCodes * (sh.m_pad2 / 2) : 0;
  z.rb_long = (size_t)grid_long * (size_t)std::max<int32_t>(P.max_long_len, 1);
  z.rb_resc = (size_t)grid_resc * (size_t)rescore_stride(P);
  return z;
}

// Launches the inter-task kernel over the short bins (a.bin_begin and the
// count are the runner's); returns SW_OK or an error code.
typedef std::function<int(InterArgs& a, int R, int W, hipStream_t s)> BinRunner;

int enqueue_search_kernels(Searcher* db, const SearchShape& sh, const SearchScratch& X,
                           const uint8_t* d_query, int32_t m, const Matrix& mat, int32_t go,
                           int32_t ge, int32_t* d_out, hipStream_t s,
                           const BinRunner* bins = nullptr);

// The searcher's own scratch for a query of this shape, grown as needed.
int reserve_search_scratch(Searcher* db, const SearchShape& sh, SearchScratch* X) {
  hipError_t e;
  const int64_t n_long = db->d->plan.n_long;
  const int64_t off_pairs = sh.off_bins > 0 ? db->d->bin_pair_end[(size_t)sh.off_bins - 1] : 0;
  const bool pairs = n_long > 0 || off_pairs > 0;
  if ((e = db->prof.reserve((size_t)sh.n_strips * prof_strip_dwords(sh.R))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("profile allocation: ") + hipGetErrorString(e));
  if ((e = db->prof2.reserve((size_t)kIntraCodes * sh.m_pad2)) != hipSuccess)
    return fail(SW_ENOMEM, std::string("profile allocation: ") + hipGetErrorString(e));
  if (pairs && (e = db->prof3.reserve((size_t)kIntraCodes * (sh.m_pad2 / 2))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("profile allocation: ") + hipGetErrorString(e));
  const int grid_long =
      (int)std::min<int64_t>(db->d->n_long_pairs + off_pairs, kIntraGridLong);
  const int grid_seg = (int)std::min<int64_t>(db->d->n_seg_items + off_pairs, kIntraGridLong);
  if (n_long > 0 && off_pairs > 0 &&
      (e = db->seg_best.reserve((size_t)(db->d->n_seg_items + off_pairs))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("long scratch: ") + hipGetErrorString(e));
  if (pairs && (e = db->rb_long.reserve(std::max<size_t>(
                    {(size_t)std::max(grid_long, 1) * (size_t)pair_stride(*db->d),
                     (size_t)grid_seg * (size_t)seg_stride(*db->d), 1}))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("long scratch: ") + hipGetErrorString(e));
  X->rb = db->rb.p;
  X->flags = db->flags.p;
  X->prof = db->prof.p;
  X->prof2 = db->prof2.p;
  X->prof3 = pairs ? db->prof3.p : nullptr;
  X->rb_long = db->rb_long.p;
  X->grid_long = grid_long;
  X->grid_seg = grid_seg;
  X->seg_best = n_long > 0 ? db->seg_best.p : nullptr;
  X->rb_resc = db->rb_resc.p;
  X->grid_resc = kIntraGridRescore;
  return SW_OK;
}

int enqueue_search(Searcher* db, const uint8_t* d_query, int32_t m, const Matrix& mat, int32_t go,
                   int32_t ge, int32_t* d_out, hipStream_t s) {
  hipError_t e;
  if (db->d->n_seqs == 0) return SW_OK;
  if (m == 0) {
    e = launch_fill(d_out, db->d->n_seqs, 0, s);
    return e == hipSuccess ? SW_OK : hip_fail(e, "fill");
  }
  const SearchShape sh = search_shape(db, m);
  SearchScratch X;
  const int rc = reserve_search_scratch(db, sh, &X);
  if (rc != SW_OK) return rc;
  return enqueue_search_kernels(db, sh, X, d_query, m, mat, go, ge, d_out, s);
}

// The kernels of one search (profile, long list, inter-task bins,
// rescoring) on stream s with the given scratch.  m > 0, n_seqs > 0.
int enqueue_search_kernels(Searcher* db, const SearchShape& sh, const SearchScratch& X,
                           const uint8_t* d_query, int32_t m, const Matrix& mat, int32_t go,
                           int32_t ge, int32_t* d_out, hipStream_t s, const BinRunner* bins) {
  hipError_t e;
  const int R = sh.R, W = sh.W, RR = sh.RR, W2 = sh.W2, RRr = sh.RRr, W2r = sh.W2r;
  const int m_pad2 = sh.m_pad2;
  const int64_t n_long = db->d->plan.n_long;
  const int n_bins = (int)db->d->plan.n_bins;
  int2* const flist = reinterpret_cast<int2*>(X.flags + 2);
  // short queries: the long pairs in column segments (seg_overlap), each
  // handed-over pair one segment; the longest short bins go to the pair
  // kernel as pairs (pick_offload; the bin runners' searches hand none over)
  const int32_t overlap = n_long > 0 ? seg_overlap(*db->d, m, mat, ge) : -1;
  const bool segmented = overlap >= 0 && X.seg_best && X.grid_seg > 0;
  const int off_bins = (int)std::min<int64_t>(std::max<int64_t>(sh.off_bins, 0), n_bins);
  const int64_t off_pairs = off_bins > 0 ? db->d->bin_pair_end[(size_t)off_bins - 1] : 0;
  const bool pairs = n_long > 0 || off_pairs > 0;

  const int t_total = time_begin(db, kTimeTotal, s);
  if ((e = launch_profile(d_query, m, mat, X.prof, sh.m_pad, R, X.prof2,
                          pairs ? X.prof3 : nullptr, m_pad2, X.flags, s)) != hipSuccess)
    return hip_fail(e, "profile kernel");
  if (pairs && (e = hipEventRecord(db->ev_fork, s)) != hipSuccess) return hip_fail(e, "event");

  IntraArgs ia{};
  ia.res = db->d->res.p;
  ia.offs = db->d->offs.p;
  ia.prof2 = X.prof2;
  ia.q0.prof2_off = 0;
  ia.q0.out_off = 0;
  ia.q0.m_pad2 = m_pad2;
  ia.queries = nullptr;
  ia.go = go;
  ia.ge = ge;
  ia.out = d_out;

  // short sequences: inter-task kernel over the bins not handed over
  auto run_bins = [&]() -> int {
    InterArgs a{};
    a.res2 = reinterpret_cast<const uint2*>(db->d->packed.p);
    a.bins = db->d->bins.p;
    a.bin_begin = off_bins;
    a.n_strips = sh.n_strips;
    a.prof = X.prof;
    a.go2 = half_pair(go);
    a.ge2 = half_pair(ge);
    a.rb = X.rb;
    a.slot_seq = db->d->slot_seq.p;
    a.out = d_out;
    a.flag_count = X.flags;
    a.flag_list = flist;
    a.sat_limit = effective_limit(db->sat_limit);
    if (bins) return (*bins)(a, R, W, s);
    if (n_bins > off_bins) {
      const int ti = time_begin(db, kTimeInter, s);
      if ((e = launch_inter(R, W, n_bins - off_bins, a, s)) != hipSuccess)
        return hip_fail(e, "inter-task kernel");
      time_end(db, ti, s);
      ++db->stats.n_inter_launches;
    }
    return SW_OK;
  };

  // long sequences (and handed-over bins): packed long-pair kernel on the
  // auxiliary stream, overlapped with the inter-task bins
  auto run_pairs = [&]() -> int {
    if (!pairs) return SW_OK;
    if ((e = hipStreamWaitEvent(db->aux_stream, db->ev_fork, 0)) != hipSuccess)
      return hip_fail(e, "stream wait");
    IntraPairArgs la{};
    la.res = db->d->res.p;
    la.offs = db->d->offs.p;
    la.items = db->d->d_long_pairs.p;
    la.count = (int32_t)(db->d->n_long_pairs + off_pairs);
    la.prof3 = X.prof3;
    la.m_pad2 = m_pad2;
    la.n_pass = (m + 64 * RR - 1) / (64 * RR);
    la.go2 = half_pair(go);
    la.ge2 = half_pair(ge);
    la.sat_limit = effective_limit(db->sat_limit);
    la.scratch = X.rb_long;
    la.scratch_stride = pair_stride(*db->d);
    la.out = d_out;
    la.flag_count = X.flags;
    la.flag_list = flist;
    int grid = std::min<int>(X.grid_long, la.count);
    if (segmented) {
      la.seg_items = db->d->d_seg_items.p;
      la.count = (int32_t)(db->d->n_seg_items + off_pairs);
      la.seg_cols = db->d->seg_cols;
      la.seg_overlap = overlap;
      la.seg_best = X.seg_best;
      la.scratch_stride = seg_stride(*db->d);
      grid = std::min<int>(X.grid_seg, la.count);
    }
    const int tl = time_begin(db, kTimeIntra, db->aux_stream);
    if ((e = launch_intra_pairs(RR, W2, grid, la, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "intra-task kernel");
    db->stats.long_items = la.count;
    db->stats.long_overlap = segmented ? overlap : -1;
    if (segmented &&
        (e = launch_long_combine(db->d->d_long_pairs.p, db->d->d_pair_seg0.p,
                                 (int32_t)(db->d->n_long_pairs + off_pairs), X.seg_best,
                                 la.sat_limit, d_out, X.flags, flist, db->aux_stream)) !=
            hipSuccess)
      return hip_fail(e, "segment maxima");
    time_end(db, tl, db->aux_stream);
    if ((e = hipEventRecord(db->ev_join, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "event");
    return SW_OK;
  };

  // The bins go first: the longest bin's workgroup is the inter-task
  // kernel's critical path and starts at once, before the long pairs' large
  // workgroups fill the CUs.  A bin runner (hybrid and allocation-free
  // searches) returns only when its bins are done, so there the pairs go first.
  int rc;
  if (bins) {
    if ((rc = run_pairs()) != SW_OK || (rc = run_bins()) != SW_OK) return rc;
  } else {
    if ((rc = run_bins()) != SW_OK || (rc = run_pairs()) != SW_OK) return rc;
  }
  // both packed kernels fill the rescoring list: join before consuming it
  if (pairs && (e = hipStreamWaitEvent(s, db->ev_join, 0)) != hipSuccess)
    return hip_fail(e, "stream wait");
  {
    // exact rescoring of sequences whose half-precision score reached the
    // limit; the workgroups read the list's length on the device
    IntraArgs ra = ia;
    ra.items = flist;
    ra.count_ptr = X.flags;
    ra.count = 0;
    ra.scratch = X.rb_resc;
    ra.scratch_stride = rescore_stride(db->d->plan);
    ra.q0.n_pass = (m + 64 * RRr - 1) / (64 * RRr);
    const int tr = time_begin(db, kTimeRescore, s);
    if ((e = launch_intra(RRr, W2r, X.grid_resc, ra, s)) != hipSuccess)
      return hip_fail(e, "rescoring kernel");
    time_end(db, tr, s);
  }
  time_end(db, t_total, s);

  db->stats.rows = R;
  db->stats.waves = W;
  const int64_t pair_res =
      db->d->long_residues + (off_bins > 0 ? db->d->bin_res_cum[(size_t)off_bins] : 0);
  db->stats.inter_cells += (int64_t)m * (db->d->n_res - pair_res);
  db->stats.intra_cells += (int64_t)m * pair_res;
  return SW_OK;
}

// The k best hits of the score row d_scores of a query just searched on
// stream s (its intra-task profile is still in db->prof2): device top-k
// selection, then the exact 32-bit intra-task kernel with end tracking over
// the k hit sequences, writing {seq, score, query end, db end} to d_hits.
int enqueue_hits(Searcher* db, int32_t m, const Matrix& mat, int32_t go, int32_t ge,
                 const int32_t* d_scores, int32_t k, sw_hit* d_hits, hipStream_t s) {
  hipError_t e;
  const int64_t n = db->d->n_seqs;
  k = (int32_t)std::min<int64_t>(k, n);
  if (k <= 0) return SW_OK;
  // the hit sequences in column segments (as the long pairs of the search:
  // windows reaching the reach of an alignment back), so a long hit no
  // longer sets the end pass's time
  const int32_t overlap = m > 0 ? hit_overlap(*db->d, m, mat, ge) : -1;
  const int32_t C = db->d->seg_cols;
  const int64_t per_hit =
      overlap >= 0 ? std::max<int64_t>(1, (db->d->plan.max_len + C - 1) / C) : 0;
  const int32_t cap = (int32_t)std::min<int64_t>((int64_t)k * per_hit, INT32_MAX);
  const size_t st_words = sizeof(TopkState) / 4;
  // state, gt[k], ties[k], items[k] (int2); with segments seg0[k + 1],
  // seg_items[cap] (int2) and, 16-byte aligned, seg_ends[cap] (int4)
  const size_t seg0_at = st_words + 4 * (size_t)k;
  const size_t sitems_at = seg0_at + (((size_t)k + 1 + 1) & ~size_t(1));
  const size_t sends_at = (sitems_at + 2 * (size_t)cap + 3) & ~size_t(3);
  const size_t words = overlap >= 0 ? sends_at + 4 * (size_t)cap : seg0_at;
  if ((e = db->topk.reserve(words)) != hipSuccess)
    return fail(SW_ENOMEM, std::string("top-k scratch: ") + hipGetErrorString(e));
  TopkState* st = reinterpret_cast<TopkState*>(db->topk.p);
  int32_t* gt = db->topk.p + st_words;
  int32_t* ties = gt + k;
  int2* items = reinterpret_cast<int2*>(ties + k);
  if ((e = launch_topk(d_scores, n, k, st, gt, ties, items, s)) != hipSuccess)
    return hip_fail(e, "top-k kernels");
  if (m == 0) {   // empty query: every score 0, no ends
    if ((e = launch_empty_hits(items, k, reinterpret_cast<int4*>(d_hits), s)) != hipSuccess)
      return hip_fail(e, "hit list");
    return SW_OK;
  }
  int RR = 8, W2 = 1;
  pick_intra(db, m, 8, &RR, &W2);
  IntraArgs ea{};
  ea.res = db->d->res.p;
  ea.offs = db->d->offs.p;
  ea.items = items;
  ea.count_ptr = nullptr;
  ea.count = k;
  ea.prof2 = db->prof2.p;
  ea.q0.prof2_off = 0;
  ea.q0.out_off = 0;
  ea.q0.m_pad2 = intra_rows_pad(m);
  ea.q0.n_pass = (m + 64 * RR - 1) / (64 * RR);
  ea.queries = nullptr;
  ea.go = go;
  ea.ge = ge;
  ea.scratch = db->rb_resc.p;
  ea.scratch_stride = rescore_stride(db->d->plan);
  ea.out = nullptr;
  ea.ends = reinterpret_cast<int4*>(d_hits);
  if (overlap >= 0) {
    int32_t* seg0 = db->topk.p + seg0_at;
    int2* seg_items = reinterpret_cast<int2*>(db->topk.p + sitems_at);
    int4* seg_ends = reinterpret_cast<int4*>(db->topk.p + sends_at);
    if ((e = launch_hit_segments(items, k, db->d->offs.p, C, cap, seg0, seg_items, s)) !=
        hipSuccess)
      return hip_fail(e, "hit segments");
    ea.seg_items = seg_items;
    ea.seg_cols = C;
    ea.seg_overlap = overlap;
    ea.count_ptr = seg0 + k;
    ea.ends = seg_ends;
    if ((e = launch_intra(RR, W2, std::min<int>(cap, kIntraGridRescore), ea, s)) != hipSuccess)
      return hip_fail(e, "hit-end kernel");
    if ((e = launch_hit_combine(items, k, seg0, seg_ends, reinterpret_cast<int4*>(d_hits), s)) !=
        hipSuccess)
      return hip_fail(e, "hit ends");
    return SW_OK;
  }
  const int grid = std::min<int>(k, kIntraGridRescore);
  if ((e = launch_intra(RR, W2, grid, ea, s)) != hipSuccess) return hip_fail(e, "hit-end kernel");
  return SW_OK;
}

// Largest magnitude a global or semi-global score may reach (the kernels'
// -infinity is -2^29).
constexpr int64_t kModeRange = int64_t(1) << 28;

// Bound on the magnitude of every value a global / semi-global search of a
// query of length m computes: gaps over every row and column of the padded
// matrix plus 128 per cell step.
int64_t mode_bound(const Searcher* db, int64_t m, int64_t go, int64_t ge) {
  return go + (ge + 128) * (m + 512 + (int64_t)db->d->plan.max_len + 1024);
}

// Global / semi-global search of one query: the int32 inter-task kernel over
// the short bins and the int32 wavefront kernel over the long list, on the
// auxiliary stream beside it.
int enqueue_search_mode(Searcher* db, const uint8_t* d_query, int32_t m, const Matrix& mat,
                        int32_t go, int32_t ge, int mode, int32_t* d_out, hipStream_t s) {
  hipError_t e;
  const Plan& P = db->d->plan;
  const int64_t n = db->d->n_seqs;
  if (n == 0) return SW_OK;
  if (m == 0) {
    if ((e = launch_mode_empty_query(db->d->offs.p, n, mode, go, ge, d_out, s)) != hipSuccess)
      return hip_fail(e, "empty-query kernel");
    return SW_OK;
  }
  // 32 rows per strip, 16 for queries of at most 16 residues: each strip
  // pays its boundary row and profile staging, so taller strips win even
  // with padding (144 residues: 5 strips of 32 beat 9 of 16; 16-row strips
  // for every query ran at 1,108 GCUPS against 1,740 with 32)
  const int R = m <= 16 ? 16 : 32;
  const int n_strips = (m + R - 1) / R;
  const int m_pad2 = intra_rows_pad(m);
  const int64_t short_dwords = P.n_bins < P.n_bins + P.n_long_bins ? P.bins[4 * P.n_bins]
                                                                  : P.packed_dwords;
  if ((e = db->mprof.reserve((size_t)n_strips * kProfRowDwords * R)) != hipSuccess ||
      (e = db->prof2.reserve((size_t)kIntraCodes * m_pad2)) != hipSuccess ||
      (e = db->rb_mode.reserve((size_t)std::max<int64_t>(4 * short_dwords, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("mode search scratch: ") + hipGetErrorString(e));
  const int t_total = time_begin(db, kTimeTotal, s);
  if ((e = launch_mode_profile(d_query, m, mat, R, n_strips, db->mprof.p, db->prof2.p, m_pad2,
                               s)) != hipSuccess)
    return hip_fail(e, "profile kernel");
  const int64_t n_long = P.n_long;
  if (n_long > 0) {
    if ((e = hipEventRecord(db->ev_fork, s)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipStreamWaitEvent(db->aux_stream, db->ev_fork, 0)) != hipSuccess)
      return hip_fail(e, "stream wait");
    int RR = 8, W2 = 1;
    pick_intra(db, m, 8, &RR, &W2);
    const int grid = (int)std::min<int64_t>(n_long, kIntraGridLong);
    if ((e = reserve_long_scratch(db, grid)) != hipSuccess)
      return fail(SW_ENOMEM, std::string("long scratch: ") + hipGetErrorString(e));
    IntraArgs la{};
    la.res = db->d->res.p;
    la.offs = db->d->offs.p;
    la.items = db->d->d_long_items.p;
    la.count = (int32_t)n_long;
    la.prof2 = db->prof2.p;
    la.q0.m_pad2 = m_pad2;
    la.q0.n_pass = (m + 64 * RR - 1) / (64 * RR);
    la.go = go;
    la.ge = ge;
    la.scratch = db->rb_long.p;
    la.scratch_stride = std::max<int64_t>(P.max_long_len, 1);
    la.out = d_out;
    la.mode = mode;
    la.m = m;
    const int tl = time_begin(db, kTimeIntra, db->aux_stream);
    if ((e = launch_intra(RR, W2, grid, la, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "intra-task kernel");
    time_end(db, tl, db->aux_stream);
    if ((e = hipEventRecord(db->ev_join, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "event");
  }
  if (P.n_bins > 0) {
    ModeArgs a{};
    a.res = db->d->packed.p;
    a.bins = db->d->bins.p;
    a.slot_seq = db->d->slot_seq.p;
    a.offs = db->d->offs.p;
    a.n_halfbins = (int32_t)(2 * P.n_bins);
    a.n_strips = n_strips;
    a.m = m;
    a.go = go;
    a.ge = ge;
    a.prof = db->mprof.p;
    a.rb = db->rb_mode.p;
    a.out = d_out;
    const int ti = time_begin(db, kTimeInter, s);
    if ((e = launch_mode_inter(R, mode, a, s)) != hipSuccess)
      return hip_fail(e, "inter-task mode kernel");
    time_end(db, ti, s);
  }
  if (n_long > 0 && (e = hipStreamWaitEvent(s, db->ev_join, 0)) != hipSuccess)
    return hip_fail(e, "stream wait");
  time_end(db, t_total, s);
  db->stats.inter_cells += (int64_t)m * (db->d->n_res - db->d->long_residues);
  db->stats.intra_cells += (int64_t)m * db->d->long_residues;
  return SW_OK;
}

// Builds (or keeps) the batch plan for these queries, matrix, gaps and
// buffers: pairs of length-sorted queries, pair and per-query descriptors,
// the (pair, half bin) work list costliest first, and the (sequence, query)
// list of long-sequence items.
int prepare_batch(Searcher* db, const uint8_t* d_queries, const int64_t* qoffs, int32_t nq,
                  const Matrix& mat, int32_t go, int32_t ge, int32_t* d_out) {
  BatchPlan& B = db->batch;
  // schedule: options, else the autotuned entry of the median query length,
  // else the one fitted to the pairs' lengths
  int R = kDefaultRows, W = kDefaultWaves;
  {
    std::vector<int64_t> lens;
    for (int32_t q = 0; q < nq; ++q)
      if (qoffs[q + 1] > qoffs[q]) lens.push_back(qoffs[q + 1] - qoffs[q]);
    std::sort(lens.begin(), lens.end(), std::greater<int64_t>());
    bool tuned = false;
    if (!lens.empty()) {
      const int b = tune_bucket((int)lens[lens.size() / 2]);
      if (db->tune_brows[b]) { R = db->tune_brows[b]; W = db->tune_bwaves[b]; tuned = true; }
    }
    if (!tuned && !lens.empty()) {
      // a pair of neighbouring lengths costs ceil(S / W) rounds of its
      // S = ceil(m / R) strips (m the longer query) for every half bin
      double best = 1e300;
      for (const Sched& c : kBatchScheds) {
        if ((db->opt_rows && c.R != db->opt_rows) || (db->opt_waves && c.W != db->opt_waves))
          continue;
        double cost = 0;
        for (size_t i = 0; i < lens.size(); i += 2) {
          const int64_t strips = (lens[i] + c.R - 1) / c.R;
          cost += (double)((strips + c.W - 1) / c.W) * c.W * c.R / c.eff;
        }
        if (cost < best) { best = cost; R = c.R; W = c.W; }
      }
    }
  }
  if (db->opt_rows == 12 || db->opt_rows == 14 || db->opt_rows == 16 || db->opt_rows == 18 ||
      db->opt_rows == 20 || db->opt_rows == 32)
    R = db->opt_rows;
  if (db->opt_waves == 4 || db->opt_waves == 8 || db->opt_waves == 12 || db->opt_waves == 16)
    W = db->opt_waves;
  if (W == 12 && R == 32) W = 8;                   // no 12-wave form of 32 rows
  if (R == 20) W = 12;                             // 20 rows: 12 waves only
  if (W == 16 && R != 12 && R != 14) R = 12;       // 16 waves: 12- or 14-row strips
  if (W != 12 && W != 16 && R != 16 && R != 32) R = 16;
  std::vector<int64_t> qv(qoffs, qoffs + nq + 1);
  if (B.valid && B.qoffs == qv && memcmp(&B.mat, &mat, sizeof(mat)) == 0 && B.go == go &&
      B.ge == ge && B.d_queries == d_queries && B.d_out == d_out && B.R == R && B.W == W &&
      B.sat_limit == db->sat_limit)
    return SW_OK;
  B.release();
  hipError_t e;
  std::vector<int32_t> order;
  std::vector<int64_t> ms(nq);
  B.zero_queries.clear();
  for (int32_t q = 0; q < nq; ++q) {
    ms[q] = qoffs[q + 1] - qoffs[q];
    if (ms[q] > 0) order.push_back(q);
    else B.zero_queries.push_back(q);
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ms[a] > ms[b]; });
  const int n_nz = (int)order.size();
  // pairs of adjacent lengths
  std::vector<PairDesc> pairs;
  int64_t prof_dw = 0;
  for (int i = 0; i < n_nz; i += 2) {
    PairDesc pd{};
    pd.qa = order[i];
    pd.qb = i + 1 < n_nz ? order[i + 1] : -1;
    pd.n_strips = (int32_t)((ms[pd.qa] + R - 1) / R);
    pd.prof_off = prof_dw;
    prof_dw += (int64_t)pd.n_strips * R * kBatchRowDwords;
    B.max_pair_work = std::max<int64_t>(B.max_pair_work, (int64_t)pd.n_strips * R * kBatchRowDwords);
    pairs.push_back(pd);
  }
  // intra-task parameters from the median query length: the 32-bit
  // kernel's (long sequences of the i32 form, rescoring) and the packed
  // long-pair kernel's
  const int64_t m_med = n_nz ? ms[order[n_nz / 2]] : 1;
  int RR = 8, W2 = 1, RRp = 8, W2p = 1;
  pick_intra(db, (int)m_med, 8, &RR, &W2);
  pick_intra(db, (int)m_med, 8, &RRp, &W2p, true);
  const int W2r = W2;
  const bool has_vlong = db->d->plan.n_vlong > 0;
  std::vector<QueryDesc> qd((size_t)std::max(nq, 1));
  int64_t prof2_bytes = 0, prof3_dw = 0;
  for (int32_t q = 0; q < nq; ++q) {
    const int64_t m = std::max<int64_t>(ms[q], 1);
    qd[q].m_pad2 = (int32_t)((m + 511) / 512 * 512);
    qd[q].n_pass = (int32_t)((m + 64 * RR - 1) / (64 * RR));
    qd[q].n_pass3 = (int32_t)((m + 64 * RRp - 1) / (64 * RRp));
    qd[q].prof2_off = prof2_bytes;
    qd[q].prof3_off = prof3_dw;
    qd[q].out_off = (int64_t)q * db->d->n_seqs;
    prof2_bytes += (int64_t)kIntraCodes * qd[q].m_pad2;
    if (has_vlong) prof3_dw += (int64_t)kIntraCodes * (qd[q].m_pad2 / 2);
    if (ms[q] > 0) B.max_query_work = std::max<int64_t>(B.max_query_work, (int64_t)kIntraCodes * qd[q].m_pad2);
  }
  // (pair, half bin) items, costliest first
  // every half bin holding at least one sequence, short and long bins
  const int64_t n_hb = 2 * (db->d->plan.n_bins + db->d->plan.n_long_bins);
  std::vector<int2> items;
  items.reserve((size_t)(n_hb * (int64_t)pairs.size()));
  for (int64_t hb = 0; hb < n_hb; ++hb) {
    if (db->d->plan.bin_count[(size_t)(hb >> 1)] <= (hb & 1)) continue;
    for (int p = 0; p < (int)pairs.size(); ++p) items.push_back(make_int2(p, (int)hb));
  }
  const std::vector<int64_t>& bins = db->d->plan.bins;
  auto cost = [&](const int2& it) {
    return (int64_t)pairs[it.x].n_strips * (bins[(size_t)(it.y >> 1) * 4 + 2] / 4 + 2 * W);
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const int2& a, const int2& b) { return cost(a) > cost(b); });
  // the very long sequences (longest first) in pairs of neighbours, and
  // (pair, query) items for the packed long-pair kernel, costliest first
  std::vector<int2> vpairs;
  for (int64_t t = 0; t < db->d->plan.n_vlong; t += 2)
    vpairs.push_back(make_int2(db->d->long_ids[(size_t)t],
                               t + 1 < db->d->plan.n_vlong ? db->d->long_ids[(size_t)t + 1] : -1));
  std::vector<int2> litems;
  for (int p = 0; p < (int)vpairs.size(); ++p)
    for (int32_t q : order) litems.push_back(make_int2(p, q));
  auto lcost = [&](const int2& it) {
    return ms[it.y] * (int64_t)db->d->long_len[(size_t)vpairs[(size_t)it.x].x];
  };
  std::stable_sort(litems.begin(), litems.end(),
                   [&](const int2& a, const int2& b) { return lcost(a) > lcost(b); });
  B.inter_cells = B.intra_cells = 0;
  for (int32_t q : order) {
    B.inter_cells += ms[q] * (db->d->n_res - db->d->vlong_residues);
    B.intra_cells += ms[q] * db->d->vlong_residues;
  }

  auto put = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  if ((e = B.pairs.reserve(std::max<size_t>(pairs.size(), 1))) != hipSuccess ||
      (e = B.qdesc.reserve(qd.size())) != hipSuccess ||
      (e = B.items.reserve(std::max<size_t>(items.size(), 1))) != hipSuccess ||
      (e = B.long_items.reserve(std::max<size_t>(litems.size(), 1))) != hipSuccess ||
      (e = B.vpairs.reserve(std::max<size_t>(vpairs.size(), 1))) != hipSuccess ||
      (e = B.prof3.reserve((size_t)std::max<int64_t>(prof3_dw, 4))) != hipSuccess ||
      (e = B.qoffs_d.reserve(qv.size())) != hipSuccess ||
      (e = B.prof.reserve((size_t)std::max<int64_t>(prof_dw, 1))) != hipSuccess ||
      (e = B.prof2.reserve((size_t)std::max<int64_t>(prof2_bytes, 16))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("batch allocation: ") + hipGetErrorString(e));
  if ((e = put(B.pairs.p, pairs.data(), pairs.size() * sizeof(PairDesc))) != hipSuccess ||
      (e = put(B.qdesc.p, qd.data(), qd.size() * sizeof(QueryDesc))) != hipSuccess ||
      (e = put(B.items.p, items.data(), items.size() * sizeof(int2))) != hipSuccess ||
      (e = put(B.long_items.p, litems.data(), litems.size() * sizeof(int2))) != hipSuccess ||
      (e = put(B.vpairs.p, vpairs.data(), vpairs.size() * sizeof(int2))) != hipSuccess ||
      (e = put(B.qoffs_d.p, qv.data(), qv.size() * sizeof(int64_t))) != hipSuccess)
    return hip_fail(e, "batch descriptors");
  B.n_pairs = (int)pairs.size();
  B.n_items = (int64_t)items.size();
  B.n_long_items = (int64_t)litems.size();
  B.R = R;
  B.W = W;
  B.RR = RR;
  B.W2 = W2;
  B.W2r = W2r;
  B.RRp = RRp;
  B.W2p = W2p;
  B.grid_b = db->d->n_cus * batch_workgroups_per_cu(R, W);
  B.grid_long = (int)std::min<int64_t>(B.n_long_items, kIntraGridLong);
  if ((e = db->rb_batch.reserve((size_t)B.grid_b * (size_t)(db->d->plan.max_all_bin_len / 4) * 128)) !=
          hipSuccess ||
      (e = db->counter.reserve(1)) != hipSuccess ||
      (e = reserve_flags(db, ((db->d->plan.n_bins + db->d->plan.n_long_bins) * (int64_t)SW_BIN_SEQS +
                              db->d->plan.n_vlong) * std::max(n_nz, 1))) != hipSuccess ||
      (e = reserve_long_scratch(db, std::max(B.grid_long, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("batch scratch: ") + hipGetErrorString(e));
  B.qoffs = qv;
  B.mat = mat;
  B.go = go;
  B.ge = ge;
  B.sat_limit = db->sat_limit;
  B.d_queries = d_queries;
  B.d_out = d_out;
  B.valid = true;
  return SW_OK;
}

// Enqueues the prepared batch on stream s (graph capture safe: kernels only).
int enqueue_batch_kernels(Searcher* db, hipStream_t s) {
  BatchPlan& B = db->batch;
  hipError_t e;
  const int64_t n = db->d->n_seqs;
  const int t_total = time_begin(db, kTimeTotal, s);
  if ((e = launch_fill(db->counter.p, 1, 0, s)) != hipSuccess ||
      (e = launch_fill(db->flags.p, 1, 0, s)) != hipSuccess)
    return hip_fail(e, "reset");
  for (int32_t q : B.zero_queries)
    if ((e = launch_fill(B.d_out + (size_t)q * n, n, 0, s)) != hipSuccess) return hip_fail(e, "fill");
  const int nq = (int)B.qoffs.size() - 1;
  if (B.n_pairs == 0) {
    time_end(db, t_total, s);
    return SW_OK;
  }
  if ((e = launch_batch_profiles(B.d_queries, B.qoffs_d.p, nq, B.mat, B.pairs.p, B.n_pairs, B.R,
                                 std::max(B.max_pair_work, B.max_query_work), B.prof.p, B.qdesc.p,
                                 B.prof2.p, B.n_long_items > 0 ? B.prof3.p : nullptr, s)) !=
      hipSuccess)
    return hip_fail(e, "batch profiles");
  IntraArgs ia{};
  ia.res = db->d->res.p;
  ia.offs = db->d->offs.p;
  ia.prof2 = B.prof2.p;
  ia.queries = B.qdesc.p;
  ia.go = B.go;
  ia.ge = B.ge;
  ia.out = B.d_out;
  // Very long sequences: the packed long-pair kernel (binary16, two
  // sequences per lane), each item with its query's profile and score row,
  // on the auxiliary stream and enqueued before the persistent batched
  // kernel, so that its workgroups take CUs first and the batched kernel's
  // fill the rest (the batched kernel holds every CU it gets until its list
  // is drained); joined before the rescoring.  Sequences at the rescoring
  // limit join the list the batched kernel fills.
  const bool vlong = B.n_long_items > 0;
  if (vlong) {
    if ((e = hipEventRecord(db->ev_fork, s)) != hipSuccess ||
        (e = hipStreamWaitEvent(db->aux_stream, db->ev_fork, 0)) != hipSuccess)
      return hip_fail(e, "stream fork");
    IntraPairArgs la{};
    la.res = db->d->res.p;
    la.offs = db->d->offs.p;
    la.items = B.vpairs.p;
    la.batch_items = B.long_items.p;
    la.queries = B.qdesc.p;
    la.count = (int32_t)B.n_long_items;
    la.prof3 = B.prof3.p;
    la.go2 = half_pair(B.go);
    la.ge2 = half_pair(B.ge);
    la.sat_limit = effective_limit(B.sat_limit);
    la.scratch = db->rb_long.p;
    la.scratch_stride = std::max<int64_t>(db->d->plan.max_long_len, 1);
    la.out = B.d_out;
    la.flag_count = db->flags.p;
    la.flag_list = flag_list(db);
    const int tl = time_begin(db, kTimeIntra, db->aux_stream);
    if ((e = launch_intra_pairs(B.RRp, B.W2p, B.grid_long, la, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "long-pair kernel");
    time_end(db, tl, db->aux_stream);
    if ((e = hipEventRecord(db->ev_join, db->aux_stream)) != hipSuccess)
      return hip_fail(e, "event");
  }
  if (db->d->plan.n_bins + db->d->plan.n_long_bins > 0) {
    BatchArgs ba{};
    ba.res = db->d->packed.p;
    ba.bins = db->d->bins.p;
    ba.items = B.items.p;
    ba.n_items = (int32_t)B.n_items;
    ba.counter = db->counter.p;
    ba.pairs = B.pairs.p;
    ba.prof = B.prof.p;
    ba.go2 = half_pair(B.go);
    ba.ge2 = half_pair(B.ge);
    ba.rb = db->rb_batch.p;
    ba.rb_stride = (int64_t)(db->d->plan.max_all_bin_len / 4) * 128;
    ba.slot_seq = db->d->slot_seq.p;
    ba.out = B.d_out;
    ba.n_seqs = n;
    ba.flag_count = db->flags.p;
    ba.flag_list = flag_list(db);
    ba.sat_limit = effective_limit(B.sat_limit);
    const int ti = time_begin(db, kTimeInter, s);
    if ((e = launch_batch(B.R, B.W, B.grid_b, ba, s)) != hipSuccess)
      return hip_fail(e, "batched inter-task kernel");
    time_end(db, ti, s);
  }
  if (vlong && (e = hipStreamWaitEvent(s, db->ev_join, 0)) != hipSuccess)
    return hip_fail(e, "stream join");
  {  // exact rescoring of what both packed kernels flagged
    IntraArgs ra = ia;
    ra.items = flag_list(db);
    ra.count_ptr = db->flags.p;
    ra.scratch = db->rb_resc.p;
    ra.scratch_stride = rescore_stride(db->d->plan);
    const int tr = time_begin(db, kTimeRescore, s);
    if ((e = launch_intra(B.RR, B.W2r, kIntraGridRescore, ra, s)) != hipSuccess)
      return hip_fail(e, "rescoring kernel");
    time_end(db, tr, s);
  }
  time_end(db, t_total, s);
  return SW_OK;
}

// Runs a batch: the kernels are captured once into a HIP graph on the
// handle's own stream and replayed while the plan stays the same; the
// caller's stream is ordered before and after with events.
int run_batch(Searcher* db, const uint8_t* d_queries, const int64_t* qoffs, int32_t nq,
              const Matrix& mat, int32_t go, int32_t ge, int32_t* d_out, hipStream_t s) {
  hipError_t e;
  if (db->d->n_seqs == 0 || nq == 0) return SW_OK;
  int rc = prepare_batch(db, d_queries, qoffs, nq, mat, go, ge, d_out);
  if (rc != SW_OK) return rc;
  BatchPlan& B = db->batch;
  hipStream_t os = db->own_stream;
  if ((e = hipEventRecord(db->ev_in, s)) != hipSuccess ||
      (e = hipStreamWaitEvent(os, db->ev_in, 0)) != hipSuccess)
    return hip_fail(e, "stream order");
  if (db->timing || !db->use_graphs) {
    rc = enqueue_batch_kernels(db, os);
    if (rc != SW_OK) return rc;
  } else {
    const void* scratch[5] = {db->rb_long.p, db->rb_resc.p, db->flags.p, db->counter.p,
                              db->rb_batch.p};
    if (B.exec && memcmp(scratch, B.captured, sizeof(scratch)) != 0) B.drop_graph();
    if (!B.exec) {
      if ((e = hipStreamBeginCapture(os, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "graph capture");
      rc = enqueue_batch_kernels(db, os);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(os, &g);
      if (rc != SW_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
      if (e != hipSuccess) return hip_fail(e, "graph capture");
      B.graph = g;
      if ((e = hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        B.drop_graph();
        return hip_fail(e, "graph instantiation");
      }
      memcpy(B.captured, scratch, sizeof(scratch));
    }
    if ((e = hipGraphLaunch(B.exec, os)) != hipSuccess) return hip_fail(e, "graph launch");
  }
  if ((e = hipEventRecord(db->ev_out, os)) != hipSuccess ||
      (e = hipStreamWaitEvent(s, db->ev_out, 0)) != hipSuccess)
    return hip_fail(e, "stream order");
  db->stats.rows = B.R;
  db->stats.waves = B.W;
  db->stats.n_inter_launches += db->d->plan.n_bins + db->d->plan.n_long_bins > 0 ? 1 : 0;
  db->stats.inter_cells += B.inter_cells;
  db->stats.intra_cells += B.intra_cells;
  return SW_OK;
}

}  // namespace
}  // namespace swdb

// ------------------------------------------------- allocation-free search
// Scratch of sw_search_async_noalloc: one array per GPU, part of the
// library's code object, so every GPU the library runs on holds it until the
// process ends.  On the host the array's name is only a stand-in; host code
// uses the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device (noalloc_setup) and kept in g_noalloc.
//
// Layout: the first kNoAllocRowBytes hold the inter-task boundary rows of one
// chunk of short bins at a time.  That part holds zeros between calls: it is
// cleared at set-up, and the last strip of every bin writes zeros back over
// its rows, as in the handle's own boundary buffer.  The rest is laid out per
// call (noalloc_layout): rescoring list, the three profiles, the rescoring
// kernel's rows and the long-sequence kernel's rows; none of it has to start
// at zero (the profile kernel clears the list's count, and the intra-task
// kernels read a boundary row only after a pass has written it).
static __device__ __align__(256) uint8_t scratch[SW_NOALLOC_SCRATCH_BYTES];

namespace swdb {
namespace {

constexpr size_t kNoAllocRowBytes = size_t(96) << 20;
static_assert(SW_NOALLOC_SCRATCH_BYTES > kNoAllocRowBytes + (size_t(1) << 20),
              "the allocation-free scratch needs room beside the boundary rows");
constexpr int kNoAllocMaxDevices = 64;

struct NoAllocDevice {
  uint8_t* ptr = nullptr;   // this device's copy of `scratch`
};
std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

// Looks up device `device`'s copy of the scratch array and clears its
// boundary-row part, once per device; the device must be current.
int noalloc_setup(int device, uint8_t** out) {
  if (device < 0 || device >= kNoAllocMaxDevices)
    return fail(SW_ERANGE, "allocation-free search: device index above 63");
  std::lock_guard<std::mutex> l(g_noalloc_mu);
  NoAllocDevice& nd = g_noalloc[device];
  if (!nd.ptr) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "scratch address");
    // a fill kernel, then wait: set-up happens once, before any search uses it
    if ((e = launch_fill(reinterpret_cast<int32_t*>(p), (int64_t)(kNoAllocRowBytes / 4), 0,
                         nullptr)) != hipSuccess ||
        (e = hipStreamSynchronize(nullptr)) != hipSuccess)
      return hip_fail(e, "scratch clear");
    nd.ptr = reinterpret_cast<uint8_t*>(p);
  }
  *out = nd.ptr;
  return SW_OK;
}

// Where one allocation-free search keeps its scratch inside the array at
// `base`, and the grids the long-list and rescoring kernels get there.
struct NoAllocLayout {
  SearchScratch X;
  size_t bytes = 0;   // end of the per-call part
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int noalloc_layout(const Searcher* db, const SearchShape& sh, uint8_t* base, NoAllocLayout* L) {
  const Plan& P = db->d->plan;
  if ((size_t)P.max_bin_len * 512 > kNoAllocRowBytes)
    return fail(SW_ERANGE, "allocation-free search: a short bin's boundary rows (" +
                               std::to_string((size_t)P.max_bin_len * 512) +
                               " bytes) exceed the 96 MiB chunk");
  const ScratchSizes z = scratch_sizes(db, sh, 0, 0);
  size_t at = kNoAllocRowBytes;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at = align256(at + bytes);
    return base + o;
  };
  L->X.rb = reinterpret_cast<uint4*>(base);
  L->X.flags = reinterpret_cast<int32_t*>(take(z.flags * 4));
  L->X.prof = reinterpret_cast<uint32_t*>(take(z.prof * 4));
  L->X.prof2 = reinterpret_cast<int8_t*>(take(z.prof2));
  L->X.prof3 = P.n_long > 0 ? reinterpret_cast<uint32_t*>(take(z.prof3 * 4)) : nullptr;
  L->X.seg_best =
      P.n_long > 0 ? reinterpret_cast<uint32_t*>(take((size_t)db->d->n_seg_items * 4)) : nullptr;
  // one boundary row per workgroup of the rescoring and long-list kernels;
  // both loop over their items, so a smaller grid only takes more rounds
  const size_t resc_row = align256((size_t)rescore_stride(P) * sizeof(int2));
  const size_t long_row =
      P.n_long > 0 ? align256((size_t)std::max<int32_t>(P.max_long_len, 1) * sizeof(int2)) : 0;
  const size_t total = (size_t)SW_NOALLOC_SCRATCH_BYTES;
  if (at + resc_row + long_row > total)
    return fail(SW_ERANGE, "allocation-free search needs " +
                               std::to_string(at + resc_row + long_row) +
                               " bytes of scratch, more than SW_NOALLOC_SCRATCH_BYTES (" +
                               std::to_string(total) + ")");
  const size_t avail = total - at;
  // rescoring (usually an empty list) gets up to an eighth of what is left,
  // the long list the rest
  size_t grid_resc = std::max<size_t>(
      1, std::min<size_t>({avail / 8 / resc_row, (size_t)kIntraGridRescore, 64}));
  while (grid_resc > 1 && grid_resc * resc_row + long_row > avail) --grid_resc;
  L->X.rb_resc = reinterpret_cast<int2*>(take(grid_resc * resc_row));
  L->X.grid_resc = (int)grid_resc;
  int grid_long = 0;
  if (P.n_long > 0) {
    const size_t left = total - at;   // >= long_row by the checks above
    grid_long = (int)std::max<size_t>(
        1, std::min<size_t>({left / long_row, (size_t)db->d->n_long_pairs, (size_t)kIntraGridLong}));
    L->X.rb_long = reinterpret_cast<int2*>(take((size_t)grid_long * long_row));
    // the same rows serve the column segments, at their shorter stride
    L->X.grid_seg = (int)std::min<size_t>(
        {(size_t)grid_long * long_row / ((size_t)seg_stride(*db->d) * sizeof(int2)),
         (size_t)db->d->n_seg_items, (size_t)kIntraGridLong});
  }
  L->X.grid_long = grid_long;
  L->bytes = at;
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
  sw_db* h = new (std::nothrow) sw_db();
  if (!h) return fail(SW_ENOMEM, "host allocation failed");
  DbData* d = &h->data;
  d->plan.check_codes = true;
  int rc = plan_layout(residues, offsets, n_seqs, long_threshold, &d->plan);
  if (rc != SW_OK) { delete h; return rc; }
  hipError_t e = hipGetDevice(&d->device);
  if (e != hipSuccess) { delete h; return hip_fail(e, "no HIP device"); }
  DeviceGuard g(d->device);
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d->device) == hipSuccess &&
        ncu > 0)
      d->n_cus = ncu;
  }
  d->n_seqs = n_seqs;
  d->n_res = offsets[n_seqs];
  const Plan& P = d->plan;
  d->long_ids.resize((size_t)P.n_long);
  d->long_len.assign((size_t)std::max<int64_t>(n_seqs, 1), 0);
  for (int64_t t = 0; t < P.n_long; ++t) {
    const int32_t sid = P.order[(size_t)t];
    const int64_t len = offsets[sid + 1] - offsets[sid];
    d->long_len[(size_t)sid] = (int32_t)len;
    d->long_ids[(size_t)t] = sid;
    d->long_residues += len;
    if (t < P.n_vlong) d->vlong_residues += len;
  }
  // host staging of the interleaved store
  std::vector<uint32_t> h_packed;
  std::vector<int64_t> h_bins;
  std::vector<int32_t> h_slots, h_long;
  try {
    h_packed.resize((size_t)P.packed_dwords);
    h_bins.resize((size_t)(P.n_bins + P.n_long_bins) * 4);
    h_slots.resize((size_t)(P.n_bins + P.n_long_bins) * SW_BIN_SEQS);
    h_long.resize((size_t)P.n_long);
  } catch (...) {
    destroy_db(h);
    return fail(SW_ENOMEM, "host staging allocation failed");
  }
  fill_layout(residues, offsets, P, h_packed.data(), h_bins.data(), h_slots.data(), h_long.data());
  std::vector<int2> h_long_items(h_long.size());
  for (size_t t = 0; t < h_long.size(); ++t) h_long_items[t] = make_int2(h_long[t], 0);
  // the packed intra-task kernel takes the long list (longest first) in
  // pairs of neighbours, so the two sequences of a pair have similar lengths
  std::vector<int2> h_long_pairs((h_long.size() + 1) / 2);
  for (size_t t = 0; t < h_long_pairs.size(); ++t)
    h_long_pairs[t] = make_int2(h_long[2 * t], 2 * t + 1 < h_long.size() ? h_long[2 * t + 1] : -1);
  d->n_long_pairs = (int64_t)h_long_pairs.size();
  // column segments of twice the long threshold (the longer sequence of a
  // pair sets its count)
  d->seg_cols = (int32_t)std::min<int64_t>(std::max<int64_t>(64, 2 * (int64_t)P.long_threshold),
                                           SW_MAX_LEN);
  std::vector<int2> h_seg_items;
  std::vector<int32_t> h_pair_seg0(h_long_pairs.size() + 1, 0);
  for (size_t p = 0; p < h_long_pairs.size(); ++p) {
    h_pair_seg0[p] = (int32_t)h_seg_items.size();
    const int64_t n_p = d->long_len[(size_t)h_long_pairs[p].x];
    const int64_t k_p = std::max<int64_t>(1, (n_p + d->seg_cols - 1) / d->seg_cols);
    if (k_p > 1) d->any_split = true;
    for (int64_t x = 0; x < k_p; ++x) h_seg_items.push_back(make_int2((int)p, (int)x));
  }
  h_pair_seg0[h_long_pairs.size()] = (int32_t)h_seg_items.size();
  d->n_seg_items = (int64_t)h_seg_items.size();
  // then the short bins' sequences in pairs of neighbours, bin by bin, each
  // pair also one whole-sequence segment item (for short queries, whose long
  // pairs run in segments)
  try {
    d->bin_pair_end.resize((size_t)P.n_bins);
    d->bin_res_cum.assign((size_t)P.n_bins + 1, 0);
    for (int64_t b = 0; b < P.n_bins; ++b) {
      const int32_t c = P.bin_count[(size_t)b];
      const int32_t* slot = &h_slots[(size_t)b * SW_BIN_SEQS];
      int64_t res_b = 0;
      for (int32_t t = 0; t < c; t += 2) {
        h_seg_items.push_back(make_int2((int)h_long_pairs.size(), 0));
        h_pair_seg0.push_back((int32_t)h_seg_items.size());
        h_long_pairs.push_back(make_int2(slot[t], t + 1 < c ? slot[t + 1] : -1));
        res_b += offsets[slot[t] + 1] - offsets[slot[t]];
        if (t + 1 < c) res_b += offsets[slot[t + 1] + 1] - offsets[slot[t + 1]];
      }
      d->bin_pair_end[(size_t)b] = (int64_t)h_long_pairs.size() - d->n_long_pairs;
      d->bin_res_cum[(size_t)b + 1] = d->bin_res_cum[(size_t)b] + res_b;
    }
  } catch (...) {
    destroy_db(h);
    return fail(SW_ENOMEM, "host staging allocation failed");
  }

  auto alloc_fail = [&](hipError_t err, const char* what) {
    destroy_db(h);
    return fail(SW_ENOMEM, std::string(what) + ": " + hipGetErrorString(err));
  };
  if ((e = d->packed.reserve((size_t)P.packed_dwords)) != hipSuccess) return alloc_fail(e, "packed");
  if ((e = d->bins.reserve((size_t)(P.n_bins + P.n_long_bins))) != hipSuccess)
    return alloc_fail(e, "bins");
  if ((e = d->slot_seq.reserve(h_slots.size())) != hipSuccess) return alloc_fail(e, "slots");
  if ((e = d->res.reserve((size_t)d->n_res)) != hipSuccess) return alloc_fail(e, "residues");
  if ((e = d->offs.reserve((size_t)n_seqs + 1)) != hipSuccess) return alloc_fail(e, "offsets");
  if ((e = d->d_long_items.reserve((size_t)P.n_long)) != hipSuccess) return alloc_fail(e, "long ids");
  if ((e = d->d_long_pairs.reserve(h_long_pairs.size())) != hipSuccess)
    return alloc_fail(e, "long pairs");
  if ((e = d->d_seg_items.reserve(h_seg_items.size())) != hipSuccess ||
      (e = d->d_pair_seg0.reserve(h_pair_seg0.size())) != hipSuccess)
    return alloc_fail(e, "long segments");
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  if ((e = up(d->packed.p, h_packed.data(), h_packed.size() * 4)) != hipSuccess ||
      (e = up(d->bins.p, h_bins.data(), h_bins.size() * 8)) != hipSuccess ||
      (e = up(d->slot_seq.p, h_slots.data(), h_slots.size() * 4)) != hipSuccess ||
      (e = up(d->res.p, residues, (size_t)d->n_res)) != hipSuccess ||
      (e = up(d->offs.p, offsets, ((size_t)n_seqs + 1) * 8)) != hipSuccess ||
      (e = up(d->d_long_items.p, h_long_items.data(), h_long_items.size() * 8)) != hipSuccess ||
      (e = up(d->d_long_pairs.p, h_long_pairs.data(), h_long_pairs.size() * 8)) != hipSuccess ||
      (e = up(d->d_seg_items.p, h_seg_items.data(), h_seg_items.size() * 8)) != hipSuccess ||
      (e = up(d->d_pair_seg0.p, h_pair_seg0.data(), h_pair_seg0.size() * 4)) != hipSuccess) {
    destroy_db(h);
    return hip_fail(e, "database upload");
  }
  try {
    d->h_res.assign(residues, residues + d->n_res);
    d->h_offs.assign(offsets, offsets + n_seqs + 1);
    d->h_bins.swap(h_bins);
    d->h_slots.swap(h_slots);
  } catch (...) {
    destroy_db(h);
    return fail(SW_ENOMEM, "host copy allocation failed");
  }
  if ((rc = init_searcher(&h->main, d)) != SW_OK) {
    std::string msg = get_error();
    destroy_db(h);
    set_error(msg);
    return rc;
  }
  {
    // set-up of the allocation-free search's scratch on this device (a
    // failure here is reported by that entry point, which retries it)
    uint8_t* na = nullptr;
    (void)noalloc_setup(d->device, &na);
  }
  *out_db = h;
  set_error("");
  return SW_OK;
}

int sw_db_load(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs, sw_db** out_db) {
  return sw_db_load_ex(residues, offsets, n_seqs, 0, out_db);
}

void sw_db_free(sw_db* h) { swdb::destroy_db(h); }

int sw_db_info(const sw_db* h, int64_t* n_seqs, int64_t* n_residues, int32_t* max_len,
               int64_t* n_long) {
  if (!h) return swdb::fail(SW_EINVAL, "db is NULL");
  const swdb::DbData* d = &h->data;
  if (n_seqs) *n_seqs = d->n_seqs;
  if (n_residues) *n_residues = d->n_res;
  if (max_len) *max_len = d->plan.max_len;
  if (n_long) *n_long = d->plan.n_long;
  return SW_OK;
}

static int impl_search_async(swdb::Searcher* db, const uint8_t* d_query, int32_t query_len, const int8_t* matrix,
                    int32_t gap_open, int32_t gap_extend, int32_t* d_out_scores,
                    void* hip_stream) {
  using namespace swdb;
  int rc = validate_search(db, d_query, query_len, matrix, gap_open, gap_extend, d_out_scores);
  if (rc != SW_OK) return rc;
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = enqueue_search(db, d_query, query_len, mat, gap_open, gap_extend, d_out_scores,
                      reinterpret_cast<hipStream_t>(hip_stream));
  mark_caller_work(db, reinterpret_cast<hipStream_t>(hip_stream));
  if (rc == SW_OK) set_error("");
  return rc;
}

static int impl_search(swdb::Searcher* db, const uint8_t* query, int32_t query_len, const int8_t* matrix,
              int32_t gap_open, int32_t gap_extend, int32_t* out_scores) {
  using namespace swdb;
  int rc = validate_search(db, query, query_len, matrix, gap_open, gap_extend, out_scores);
  if (rc != SW_OK) return rc;
  for (int32_t i = 0; i < query_len; ++i)
    if (query[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24 at position " + std::to_string(i));
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  hipError_t e;
  if ((e = db->q_stage.reserve((size_t)std::max(query_len, 1))) != hipSuccess ||
      (e = db->out_stage.reserve((size_t)std::max<int64_t>(db->d->n_seqs, 1))) != hipSuccess)
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
  if (db->d->n_seqs > 0 &&
      (e = hipMemcpyAsync(out_scores, db->out_stage.p, (size_t)db->d->n_seqs * 4, hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    return hip_fail(e, "score download");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
  set_error("");
  return SW_OK;
}

namespace swdb {
namespace {

// Device bytes of traceback codes per launch: the sequences are taken in
// groups whose codes fit (one sequence alone may have up to kTraceMaxBox).
constexpr int64_t kTraceGroupBytes = int64_t(1) << 30;
constexpr int64_t kTraceMaxBox = int64_t(4) << 30;

}  // namespace
}  // namespace swdb

static int impl_traceback(swdb::Searcher* db, const uint8_t* query, int32_t query_len,
                          const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                          const int32_t* seqs, int32_t n_items, sw_alignment* out, uint32_t* ops,
                          int64_t ops_cap, int64_t* ops_used) {
  using namespace swdb;
  int rc = validate_search(db, query, query_len, matrix, gap_open, gap_extend, matrix);
  if (rc != SW_OK) return rc;
  if (n_items < 0 || n_items > SW_MAX_TOPK)
    return fail(SW_ERANGE, "n_items must be 0..SW_MAX_TOPK");
  if (n_items > 0 && (!seqs || !out)) return fail(SW_EINVAL, "seqs or out is NULL");
  if (ops_cap < 0 || (ops_cap > 0 && !ops)) return fail(SW_EINVAL, "ops is NULL or ops_cap < 0");
  const int64_t n_seqs = db->d->n_seqs;
  for (int32_t t = 0; t < n_items; ++t)
    if (seqs[t] < 0 || seqs[t] >= n_seqs)
      return fail(SW_EINVAL, "sequence index out of range at item " + std::to_string(t));
  for (int32_t i = 0; i < query_len; ++i)
    if (query[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24 at position " + std::to_string(i));
  const int64_t ld = intra_rows_pad(std::max(query_len, 1));
  const std::vector<int64_t>& offs = db->d->h_offs;
  for (int32_t t = 0; t < n_items; ++t) {
    const int64_t box = (offs[(size_t)seqs[t] + 1] - offs[(size_t)seqs[t]]) * ld;
    if (box > kTraceMaxBox)
      return fail(SW_ERANGE, "traceback codes of sequence " + std::to_string(seqs[t]) + " (" +
                                 std::to_string(box) + " bytes) exceed 4 GiB");
  }
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  std::vector<int4> ends((size_t)n_items);
  std::vector<std::vector<uint32_t>> runs((size_t)n_items);
  std::vector<int32_t> qb((size_t)n_items, -1), dbb((size_t)n_items, -1);
  hipError_t e;
  hipStream_t s = db->own_stream;
  if (query_len == 0 || n_items == 0) {
    for (int32_t t = 0; t < n_items; ++t) ends[(size_t)t] = make_int4(seqs[t], 0, -1, -1);
  } else {
    int RR = 8, W2 = 1;
    pick_intra(db, query_len, 8, &RR, &W2);
    if ((e = db->q_stage.reserve((size_t)query_len)) != hipSuccess ||
        (e = db->prof2.reserve((size_t)kIntraCodes * ld)) != hipSuccess)
      return fail(SW_ENOMEM, std::string("traceback scratch: ") + hipGetErrorString(e));
    if ((e = hipMemcpyAsync(db->q_stage.p, query, (size_t)query_len, hipMemcpyHostToDevice, s)) !=
        hipSuccess)
      return hip_fail(e, "query upload");
    Matrix mat;
    memcpy(mat.v, matrix, sizeof(mat.v));
    if ((e = launch_mode_profile(db->q_stage.p, query_len, mat, 16, 0, nullptr, db->prof2.p,
                                 (int)ld, s)) != hipSuccess)
      return hip_fail(e, "traceback profile");
    std::vector<uint8_t> h_dir;
    int32_t t0 = 0;
    while (t0 < n_items) {
      // a group: as many sequences as fit kTraceGroupBytes (at least one)
      int32_t t1 = t0;
      int64_t bytes = 0;
      std::vector<int64_t> off;
      std::vector<int2> items;
      while (t1 < n_items) {
        const int64_t box = (offs[(size_t)seqs[t1] + 1] - offs[(size_t)seqs[t1]]) * ld;
        if (t1 > t0 && bytes + box > kTraceGroupBytes) break;
        off.push_back(bytes);
        items.push_back(make_int2(seqs[t1], 0));
        bytes += box;
        ++t1;
      }
      const int32_t k = t1 - t0;
      if ((e = db->trace_dir.reserve((size_t)std::max<int64_t>(bytes, 8))) != hipSuccess ||
          (e = db->trace_items.reserve((size_t)k)) != hipSuccess ||
          (e = db->trace_off.reserve((size_t)k)) != hipSuccess ||
          (e = db->trace_ends.reserve((size_t)k)) != hipSuccess)
        return fail(SW_ENOMEM, std::string("traceback codes: ") + hipGetErrorString(e));
      if ((e = hipMemcpyAsync(db->trace_items.p, items.data(), (size_t)k * sizeof(int2),
                              hipMemcpyHostToDevice, s)) != hipSuccess ||
          (e = hipMemcpyAsync(db->trace_off.p, off.data(), (size_t)k * sizeof(int64_t),
                              hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "traceback items");
      IntraArgs ta{};
      ta.res = db->d->res.p;
      ta.offs = db->d->offs.p;
      ta.items = db->trace_items.p;
      ta.count_ptr = nullptr;
      ta.count = k;
      ta.prof2 = db->prof2.p;
      ta.q0.prof2_off = 0;
      ta.q0.out_off = 0;
      ta.q0.m_pad2 = (int32_t)ld;
      ta.q0.n_pass = (query_len + 64 * RR - 1) / (64 * RR);
      ta.queries = nullptr;
      ta.go = gap_open;
      ta.ge = gap_extend;
      ta.scratch = db->rb_resc.p;
      ta.scratch_stride = rescore_stride(db->d->plan);
      ta.out = nullptr;
      ta.ends = db->trace_ends.p;
      ta.dir = db->trace_dir.p;
      ta.dir_off = db->trace_off.p;
      ta.dir_ld = ld;
      if ((e = launch_intra(RR, W2, std::min<int>(k, kIntraGridRescore), ta, s)) != hipSuccess)
        return hip_fail(e, "traceback kernel");
      if ((e = hipMemcpyAsync(ends.data() + t0, db->trace_ends.p, (size_t)k * sizeof(int4),
                              hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "traceback download");
      // of each sequence's codes only the columns the walk can visit (up to
      // the end's), one contiguous copy per sequence (a strided copy to
      // pageable memory goes column by column and took ~2 ms per sequence)
      std::vector<int64_t> hld((size_t)k, ld), hoff((size_t)k, 0);
      int64_t hbytes = 0;
      for (int32_t x = 0; x < k; ++x) {
        const int4 en = ends[(size_t)(t0 + x)];
        hoff[(size_t)x] = hbytes;
        if (en.y > 0) hbytes += ld * ((int64_t)en.w + 1);
      }
      try {
        h_dir.resize((size_t)std::max<int64_t>(hbytes, 1));
      } catch (...) {
        return fail(SW_ENOMEM, "host allocation failed");
      }
      for (int32_t x = 0; x < k; ++x) {
        const int4 en = ends[(size_t)(t0 + x)];
        if (en.y <= 0) continue;
        if ((e = hipMemcpyAsync(h_dir.data() + hoff[(size_t)x], db->trace_dir.p + off[(size_t)x],
                                (size_t)(ld * ((int64_t)en.w + 1)), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
          return hip_fail(e, "traceback download");
      }
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "traceback download");
      // the walks, one host thread per sequence of the group
      std::atomic<int32_t> next{0};
      std::atomic<bool> bad{false};
      auto work = [&]() {
        for (int32_t x; (x = next.fetch_add(1)) < k;) {
          const int4 en = ends[(size_t)(t0 + x)];
          if (en.y <= 0) continue;
          if (!walk_alignment(h_dir.data() + hoff[(size_t)x], hld[(size_t)x], en.z, en.w,
                              &qb[(size_t)(t0 + x)], &dbb[(size_t)(t0 + x)],
                              &runs[(size_t)(t0 + x)]))
            bad = true;
        }
      };
      const int nt = std::max(1, std::min<int>(k, (int)std::thread::hardware_concurrency()));
      std::vector<std::thread> pool;
      try {
        for (int x = 1; x < nt; ++x) pool.emplace_back(work);
      } catch (...) {
      }
      work();
      for (auto& th : pool) th.join();
      if (bad) return fail(SW_EDEVICE, "traceback codes do not form a path");
      t0 = t1;
    }
  }
  int64_t total = 0;
  for (const auto& r : runs) total += (int64_t)r.size();
  if (ops_used) *ops_used = total;
  if (total > ops_cap)
    return fail(SW_ERANGE, "the alignments take " + std::to_string(total) +
                               " operation runs, more than ops_cap (" + std::to_string(ops_cap) + ")");
  int64_t at = 0;
  for (int32_t t = 0; t < n_items; ++t) {
    const int4 en = ends[(size_t)t];
    sw_alignment& A = out[t];
    A.seq = seqs[t];
    A.score = std::max(en.y, 0);
    A.query_begin = en.y > 0 ? qb[(size_t)t] : -1;
    A.query_end = en.y > 0 ? en.z : -1;
    A.db_begin = en.y > 0 ? dbb[(size_t)t] : -1;
    A.db_end = en.y > 0 ? en.w : -1;
    A.ops_offset = at;
    A.n_ops = (int32_t)runs[(size_t)t].size();
    A.reserved = 0;
    if (A.n_ops > 0) memcpy(ops + at, runs[(size_t)t].data(), (size_t)A.n_ops * 4);
    at += A.n_ops;
  }
  set_error("");
  return SW_OK;
}

static int impl_search_topk_async(swdb::Searcher* db, const uint8_t* d_query, int32_t query_len,
                                  const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                                  int32_t k, int32_t* d_out_scores, sw_hit* d_hits,
                                  void* hip_stream) {
  using namespace swdb;
  int rc = validate_search(db, d_query, query_len, matrix, gap_open, gap_extend, d_out_scores);
  if (rc != SW_OK) return rc;
  if (k < 0) return fail(SW_EINVAL, "k < 0");
  if (k > SW_MAX_TOPK) return fail(SW_ERANGE, "k > SW_MAX_TOPK");
  if (k > 0 && db->d->n_seqs > 0 && !d_hits) return fail(SW_EINVAL, "hits is NULL");
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  rc = enqueue_search(db, d_query, query_len, mat, gap_open, gap_extend, d_out_scores, s);
  if (rc == SW_OK)
    rc = enqueue_hits(db, query_len, mat, gap_open, gap_extend, d_out_scores, k, d_hits, s);
  mark_caller_work(db, s);
  if (rc == SW_OK) set_error("");
  return rc;
}

static int impl_search_topk(swdb::Searcher* db, const uint8_t* query, int32_t query_len,
                            const int8_t* matrix, int32_t gap_open, int32_t gap_extend, int32_t k,
                            int32_t* out_scores, sw_hit* out_hits) {
  using namespace swdb;
  // out_scores may be NULL here: pass any non-null pointer to the check
  int rc = validate_search(db, query, query_len, matrix, gap_open, gap_extend, matrix);
  if (rc != SW_OK) return rc;
  if (k < 0) return fail(SW_EINVAL, "k < 0");
  if (k > SW_MAX_TOPK) return fail(SW_ERANGE, "k > SW_MAX_TOPK");
  const int64_t n = db->d->n_seqs;
  const int32_t kk = (int32_t)std::min<int64_t>(k, n);
  if (kk > 0 && !out_hits) return fail(SW_EINVAL, "out_hits is NULL");
  for (int32_t i = 0; i < query_len; ++i)
    if (query[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24 at position " + std::to_string(i));
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  hipError_t e;
  if ((e = db->q_stage.reserve((size_t)std::max(query_len, 1))) != hipSuccess ||
      (e = db->out_stage.reserve((size_t)std::max<int64_t>(n, 1))) != hipSuccess ||
      (e = db->hits_stage.reserve((size_t)std::max(kk, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("staging allocation: ") + hipGetErrorString(e));
  hipStream_t s = db->own_stream;
  if (query_len > 0 &&
      (e = hipMemcpyAsync(db->q_stage.p, query, (size_t)query_len, hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return hip_fail(e, "query upload");
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = enqueue_search(db, db->q_stage.p, query_len, mat, gap_open, gap_extend, db->out_stage.p, s);
  if (rc == SW_OK)
    rc = enqueue_hits(db, query_len, mat, gap_open, gap_extend, db->out_stage.p, kk,
                      reinterpret_cast<sw_hit*>(db->hits_stage.p), s);
  if (rc != SW_OK) {
    (void)hipStreamSynchronize(s);
    return rc;
  }
  if (out_scores && n > 0 &&
      (e = hipMemcpyAsync(out_scores, db->out_stage.p, (size_t)n * 4, hipMemcpyDeviceToHost, s)) !=
          hipSuccess)
    return hip_fail(e, "score download");
  if (kk > 0 && (e = hipMemcpyAsync(out_hits, db->hits_stage.p, (size_t)kk * sizeof(sw_hit),
                                    hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "hit download");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
  set_error("");
  return SW_OK;
}

// ------------------------------------------------------------ hybrid search
constexpr int64_t kHybridMinChunk = 32;   // bins per later GPU launch, at least

// The hybrid search's shared work order is the short bins' slots in
// length-sorted order (slot k of bin b is position 128 b + k).  The GPU
// takes whole bins from the front in chunks; the host threads take single
// sequences from the back (the shortest first).  The two may overlap in the
// bin where they meet (a sequence scored by both sides gets the same exact
// score).  The split is planned from measured rates: the GPU's first chunk
// leaves the host about twice the share its speed suggests, and a host
// thread only keeps a sequence it expects to finish before the planned end;
// a sequence given back (and every longer one) goes to the GPU.  When the
// GPU has no bin left it stops the host threads, waits for their current
// sequences and launches one last chunk for any bin a given-back sequence
// lies in, so every slot is scored by at least one side.
static int impl_search_hybrid(swdb::Searcher* db, const uint8_t* query, int32_t query_len,
                              const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                              int32_t cpu_threads, int32_t* out_scores, sw_hybrid_stats* hst) {
  using namespace swdb;
  using clock = std::chrono::steady_clock;
  int rc = validate_search(db, query, query_len, matrix, gap_open, gap_extend, out_scores);
  if (rc != SW_OK) return rc;
  if (cpu_threads < 0 || cpu_threads > 1024) return fail(SW_EINVAL, "cpu_threads must be 0..1024");
  for (int32_t i = 0; i < query_len; ++i)
    if (query[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24 at position " + std::to_string(i));
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  const DbData& D = *db->d;
  const int64_t n = D.n_seqs, n_bins = D.plan.n_bins;
  sw_hybrid_stats st{};
  const auto t0 = clock::now();
  const int threads = cpu_threads > 0 ? cpu_threads
                                      : std::max(1, (int)std::thread::hardware_concurrency() - 1);
  st.cpu_threads = threads;
  if (n == 0 || query_len == 0) {
    if (n > 0) memset(out_scores, 0, (size_t)n * 4);
    if (hst) *hst = st;
    set_error("");
    return SW_OK;
  }
  hipError_t e;
  if ((e = db->q_stage.reserve((size_t)query_len)) != hipSuccess ||
      (e = db->out_stage.reserve((size_t)n)) != hipSuccess)
    return fail(SW_ENOMEM, std::string("staging allocation: ") + hipGetErrorString(e));
  std::vector<int64_t> cum;   // cells of the bins before bin b, b = 0 .. n_bins
  cpu::Profile prof;
  try {
    cum.resize((size_t)n_bins + 1);
    for (int64_t b = 0; b <= n_bins; ++b) cum[(size_t)b] = D.bin_res_cum[(size_t)b] * query_len;
    cpu::build_profile(query, query_len, matrix, &prof);
  } catch (...) {
    return fail(SW_ENOMEM, "host allocation failed");
  }
  hipStream_t s = db->own_stream;
  if ((e = hipMemcpyAsync(db->q_stage.p, query, (size_t)query_len, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return hip_fail(e, "query upload");
  // every short bin takes part in the split (none handed to the long-pair
  // kernel): the host takes sequences from the back of the same order
  SearchShape sh = search_shape(db, query_len);
  sh.off_bins = 0;
  SearchScratch X;
  if ((rc = reserve_search_scratch(db, sh, &X)) != SW_OK) return rc;

  // the plan: expected time of the short bins with both sides working, the
  // host's expected share, and the deadline by which a host thread must be
  // done with anything it takes
  const double cells_all = (double)cum[(size_t)n_bins];
  const double r_gpu = db->hyb_gpu_rate, r_cpu = db->hyb_cpu_rate;
  const double t_plan = cells_all / (r_gpu + threads * r_cpu);
  const double host_share = db->hyb_share > 0 ? cells_all * db->hyb_share / 2000.0
                                              : threads * r_cpu * t_plan;
  // a fixed share (SW_OPT_HYBRID_SHARE) has no deadline: the host keeps
  // what it takes
  const auto deadline = db->hyb_share > 0 ? clock::time_point::max()
                                          : t0 + std::chrono::duration_cast<clock::duration>(
                                                     std::chrono::duration<double>(t_plan));
  const int64_t first_cells = (int64_t)std::max(0.0, cells_all - 2.0 * host_share);
  std::atomic<int64_t> back{n_bins * SW_BIN_SEQS};   // host: the next slot is back - 1
  std::atomic<int64_t> front{0};                      // GPU: the next bin
  std::atomic<int64_t> given_back{0};                 // 1 + the highest slot given back
  std::atomic<bool> gpu_done{false};
  std::atomic<int64_t> cpu_cells{0}, cpu_seqs{0};
  std::atomic<int64_t> cpu_ns{0};
  // each host thread's {sequence, score} results, applied after the GPU's
  std::vector<std::vector<int2>> host_res((size_t)threads);
  auto worker = [&](int t) {
    cpu::Workspace w;
    std::vector<int2>& mine = host_res[(size_t)t];
    int64_t cells = 0, seqs = 0, ns = 0;
    while (!gpu_done.load(std::memory_order_relaxed)) {
      const int64_t slot = back.fetch_sub(1) - 1;
      // the bins the GPU has taken stay with it
      if (slot < front.load() * SW_BIN_SEQS) break;
      const int64_t b = slot / SW_BIN_SEQS;
      const int32_t sid = D.h_slots[(size_t)(D.h_bins[(size_t)b * 4 + 3] + slot % SW_BIN_SEQS)];
      if (sid < 0) continue;
      const int64_t at = D.h_offs[(size_t)sid];
      const int len = (int)(D.h_offs[(size_t)sid + 1] - at);
      const int64_t c = (int64_t)len * query_len;
      const auto now = clock::now();
      if (deadline != clock::time_point::max() &&
          now + std::chrono::duration_cast<clock::duration>(std::chrono::duration<double>(c / r_cpu)) >
              deadline) {
        // not this one: leave it (and the longer rest) to the GPU
        int64_t top = given_back.load();
        while (top < slot + 1 && !given_back.compare_exchange_weak(top, slot + 1)) {
        }
        gpu_done = true;          // stops the other host threads too
        break;
      }
      mine.push_back(make_int2(sid, cpu::score(prof, D.h_res.data() + at, len, gap_open,
                                               gap_extend, &w)));
      ns += std::chrono::duration_cast<std::chrono::nanoseconds>(clock::now() - now).count();
      cells += c;
      ++seqs;
    }
    cpu_cells += cells;
    cpu_seqs += seqs;
    cpu_ns += ns;
  };
  bool host_started = false;
  try {
    if (!db->hpool) db->hpool.reset(new HostPool());
    db->hpool->run(threads, worker);
    host_started = true;
  } catch (...) {
    gpu_done = true;   // no host work (threads already started run and end)
    if (db->hpool && !db->hpool->threads.empty()) {
      db->hpool->run(0, [](int) {});
      host_started = true;
    }
  }
  int64_t gpu_bins = 0;
  auto t_gpu0 = clock::now(), t_gpu1 = t_gpu0;
  // first bin the GPU does not need to take: every slot from there on is
  // held by a host thread (bins a host thread has started or given a slot
  // back in are taken too)
  auto gpu_end = [&]() {
    const int64_t to = std::max<int64_t>({back.load(), given_back.load(), 0});
    return (to + SW_BIN_SEQS - 1) / SW_BIN_SEQS;
  };
  bool joined = false;
  BinRunner runner = [&](InterArgs& a, int R, int W, hipStream_t st_) -> int {
    int k = 0;
    t_gpu0 = clock::now();
    for (;;) {
      const int64_t b0 = front.load();
      int64_t end = gpu_end();
      if (end <= b0 && !joined) {
        // nothing left for the GPU: stop the host threads, wait for their
        // current sequences, and look again
        gpu_done = true;
        if (host_started) db->hpool->wait();
        joined = true;
        end = gpu_end();
      }
      const int64_t rem = end - b0;
      if (rem <= 0) break;
      int64_t take;
      if (k == 0) {   // most of the work at once, leaving the host's planned share
        take = std::upper_bound(cum.begin() + b0, cum.begin() + end + 1, first_cells) -
               (cum.begin() + b0) - 1;
        take = std::max<int64_t>(take, std::min(rem, kHybridMinChunk));
      } else {
        take = std::min(rem, std::max(kHybridMinChunk, rem / 4));
      }
      take = std::min(take, rem);
      front.store(b0 + take);
      a.bin_begin = (int32_t)b0;
      hipError_t err;
      if ((err = launch_inter(R, W, (int)take, a, st_)) != hipSuccess)
        return hip_fail(err, "inter-task kernel");
      if ((err = hipEventRecord(db->ev_chunk[k & 1], st_)) != hipSuccess)
        return hip_fail(err, "event");
      // keep at most two chunks queued: claim the next once the earlier ends
      if (k > 0 && (err = hipEventSynchronize(db->ev_chunk[(k - 1) & 1])) != hipSuccess)
        return hip_fail(err, "chunk wait");
      ++db->stats.n_inter_launches;
      gpu_bins += take;
      ++k;
    }
    if (k > 0 && hipEventSynchronize(db->ev_chunk[(k - 1) & 1]) != hipSuccess)
      (void)hipGetLastError();   // reported by the stream synchronisation below
    t_gpu1 = clock::now();
    gpu_done = true;
    return SW_OK;
  };
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = enqueue_search_kernels(db, sh, X, db->q_stage.p, query_len, mat, gap_open, gap_extend,
                              db->out_stage.p, s, &runner);
  gpu_done = true;
  if (!joined && host_started) db->hpool->wait();
  // the GPU's scores straight into the caller's array, then the host's on
  // top: the GPU scored the bins it took and the long list, a host thread
  // every slot outside the GPU's bins (and perhaps some inside, with the
  // same scores), so every entry ends up written by a side that scored it
  if (rc == SW_OK &&
      (e = hipMemcpyAsync(out_scores, db->out_stage.p, (size_t)n * 4, hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    rc = hip_fail(e, "score download");
  if ((e = hipStreamSynchronize(s)) != hipSuccess && rc == SW_OK) rc = hip_fail(e, "search");
  if (rc != SW_OK) return rc;
  for (const auto& mine : host_res)
    for (const int2& r : mine) out_scores[r.x] = r.y;
  // running averages of both sides' rates for the next plan
  const double gpu_s = std::chrono::duration<double>(t_gpu1 - t_gpu0).count();
  const double gpu_short = cells_all - (double)cpu_cells.load();
  if (gpu_s > 0 && gpu_short > 0) db->hyb_gpu_rate = 0.5 * db->hyb_gpu_rate + 0.5 * gpu_short / gpu_s;
  if (cpu_ns.load() > 0 && cpu_cells.load() > 0)
    db->hyb_cpu_rate = 0.5 * db->hyb_cpu_rate + 0.5 * (double)cpu_cells.load() / (cpu_ns.load() * 1e-9);
  st.gpu_bins = gpu_bins;
  st.cpu_seqs = cpu_seqs.load();
  st.cpu_cells = cpu_cells.load();
  st.gpu_cells = (int64_t)query_len * D.n_res - st.cpu_cells;
  st.ms = std::chrono::duration<float, std::milli>(clock::now() - t0).count();
  if (hst) *hst = st;
  set_error("");
  return SW_OK;
}

static int validate_mode(const swdb::Searcher* db, int32_t m, int32_t go, int32_t ge,
                         int32_t mode) {
  using namespace swdb;
  if (mode != SW_MODE_LOCAL && mode != SW_MODE_GLOBAL && mode != SW_MODE_SEMIGLOBAL)
    return fail(SW_EINVAL, "mode must be SW_MODE_LOCAL, SW_MODE_GLOBAL or SW_MODE_SEMIGLOBAL");
  if (mode != SW_MODE_LOCAL && mode_bound(db, m, go, ge) > kModeRange)
    return fail(SW_ERANGE, "gap penalties and lengths too large for 32-bit global scores");
  return SW_OK;
}

static int impl_search_mode_async(swdb::Searcher* db, const uint8_t* d_query, int32_t query_len,
                                  const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                                  int32_t mode, int32_t* d_out_scores, void* hip_stream) {
  using namespace swdb;
  int rc = validate_search(db, d_query, query_len, matrix, gap_open, gap_extend, d_out_scores);
  if (rc == SW_OK) rc = validate_mode(db, query_len, gap_open, gap_extend, mode);
  if (rc != SW_OK) return rc;
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  rc = mode == SW_MODE_LOCAL
           ? enqueue_search(db, d_query, query_len, mat, gap_open, gap_extend, d_out_scores, s)
           : enqueue_search_mode(db, d_query, query_len, mat, gap_open, gap_extend, mode,
                                 d_out_scores, s);
  mark_caller_work(db, s);
  if (rc == SW_OK) set_error("");
  return rc;
}

static int impl_search_mode(swdb::Searcher* db, const uint8_t* query, int32_t query_len,
                            const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                            int32_t mode, int32_t* out_scores) {
  using namespace swdb;
  int rc = validate_search(db, query, query_len, matrix, gap_open, gap_extend, out_scores);
  if (rc == SW_OK) rc = validate_mode(db, query_len, gap_open, gap_extend, mode);
  if (rc != SW_OK) return rc;
  for (int32_t i = 0; i < query_len; ++i)
    if (query[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24 at position " + std::to_string(i));
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  hipError_t e;
  if ((e = db->q_stage.reserve((size_t)std::max(query_len, 1))) != hipSuccess ||
      (e = db->out_stage.reserve((size_t)std::max<int64_t>(db->d->n_seqs, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("staging allocation: ") + hipGetErrorString(e));
  hipStream_t s = db->own_stream;
  if (query_len > 0 &&
      (e = hipMemcpyAsync(db->q_stage.p, query, (size_t)query_len, hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return hip_fail(e, "query upload");
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = mode == SW_MODE_LOCAL
           ? enqueue_search(db, db->q_stage.p, query_len, mat, gap_open, gap_extend,
                            db->out_stage.p, s)
           : enqueue_search_mode(db, db->q_stage.p, query_len, mat, gap_open, gap_extend, mode,
                                 db->out_stage.p, s);
  if (rc != SW_OK) {
    (void)hipStreamSynchronize(s);
    return rc;
  }
  if (db->d->n_seqs > 0 &&
      (e = hipMemcpyAsync(out_scores, db->out_stage.p, (size_t)db->d->n_seqs * 4,
                          hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "score download");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
  set_error("");
  return SW_OK;
}

static int impl_search_async_noalloc(swdb::Searcher* db, const uint8_t* d_query,
                                     int32_t query_len, const int8_t* matrix, int32_t gap_open,
                                     int32_t gap_extend, int32_t* d_out_scores,
                                     void* hip_stream) {
  using namespace swdb;
  int rc = validate_search(db, d_query, query_len, matrix, gap_open, gap_extend, d_out_scores);
  if (rc != SW_OK) return rc;
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  uint8_t* base = nullptr;
  if ((rc = noalloc_setup(db->d->device, &base)) != SW_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const DbData& D = *db->d;
  hipError_t e;
  if (D.n_seqs == 0) {
    set_error("");
    return SW_OK;
  }
  if (query_len == 0) {
    if ((e = launch_fill(d_out_scores, D.n_seqs, 0, s)) != hipSuccess) return hip_fail(e, "fill");
    mark_caller_work(db, s);
    set_error("");
    return SW_OK;
  }
  // no bins handed to the long-pair kernel: its boundary rows here are
  // sized for the long list only
  SearchShape sh = search_shape(db, query_len);
  sh.off_bins = 0;
  NoAllocLayout L;
  if ((rc = noalloc_layout(db, sh, base, &L)) != SW_OK) return rc;
  // the short bins in chunks whose boundary rows fit the 96 MiB part; each
  // chunk's rows start at the array's start (rb_base = the chunk's first
  // rb_off), and launches on one stream run one after the other
  const int64_t* hb = D.h_bins.data();   // {res_off, rb_off, len, slot0} per bin
  const int64_t n_bins = D.plan.n_bins;
  BinRunner runner = [&](InterArgs& a, int R, int W, hipStream_t st) -> int {
    for (int64_t b0 = 0; b0 < n_bins;) {
      const int64_t first = hb[4 * b0 + 1];
      int64_t b1 = b0 + 1;
      while (b1 < n_bins &&
             (size_t)(hb[4 * b1 + 1] + 32 * hb[4 * b1 + 2] - first) * sizeof(uint4) <=
                 kNoAllocRowBytes)
        ++b1;
      a.bin_begin = (int32_t)b0;
      a.rb = L.X.rb;
      a.rb_base = first;
      hipError_t err;
      if ((err = launch_inter(R, W, (int)(b1 - b0), a, st)) != hipSuccess)
        return hip_fail(err, "inter-task kernel");
      ++db->stats.n_inter_launches;
      b0 = b1;
    }
    return SW_OK;
  };
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  // no timing events here: recording them may create events
  const bool timing = db->timing;
  db->timing = false;
  rc = enqueue_search_kernels(db, sh, L.X, d_query, query_len, mat, gap_open, gap_extend,
                              d_out_scores, s, &runner);
  db->timing = timing;
  mark_caller_work(db, s);
  if (rc == SW_OK) set_error("");
  return rc;
}

static int validate_batch(const swdb::Searcher* db, const void* queries, const int64_t* qoffs, int32_t nq,
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
  if (nq > 0 && db->d->n_seqs > 0 && !out) return fail(SW_EINVAL, "out_scores is NULL");
  if (ge < 0 || go < ge) return fail(SW_EINVAL, "gaps must satisfy 0 <= gap_extend <= gap_open");
  if (go > SW_MAX_GAP) return fail(SW_ERANGE, "gap_open > 2^30");
  return SW_OK;
}

static int impl_search_batch_async(swdb::Searcher* db, const uint8_t* d_queries, const int64_t* query_offsets,
                          int32_t n_queries, const int8_t* matrix, int32_t gap_open,
                          int32_t gap_extend, int32_t* d_out_scores, void* hip_stream) {
  using namespace swdb;
  int rc = validate_batch(db, d_queries, query_offsets, n_queries, matrix, gap_open, gap_extend,
                          d_out_scores);
  if (rc != SW_OK) return rc;
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = run_batch(db, d_queries, query_offsets, n_queries, mat, gap_open, gap_extend, d_out_scores,
                 reinterpret_cast<hipStream_t>(hip_stream));
  mark_caller_work(db, reinterpret_cast<hipStream_t>(hip_stream));
  if (rc == SW_OK) set_error("");
  return rc;
}

static int impl_search_batch(swdb::Searcher* db, const uint8_t* queries, const int64_t* query_offsets,
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
  DeviceGuard g(db->d->device);
  hipError_t e;
  hipStream_t s = db->own_stream;
  const size_t out_n = (size_t)n_queries * (size_t)db->d->n_seqs;
  if ((e = db->q_stage.reserve((size_t)std::max<int64_t>(total, 1))) != hipSuccess ||
      (e = db->out_stage.reserve(std::max<size_t>(out_n, 1))) != hipSuccess)
    return fail(SW_ENOMEM, std::string("staging allocation: ") + hipGetErrorString(e));
  if (total > 0 &&
      (e = hipMemcpyAsync(db->q_stage.p, queries, (size_t)total, hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return hip_fail(e, "query upload");
  Matrix mat;
  memcpy(mat.v, matrix, sizeof(mat.v));
  rc = run_batch(db, db->q_stage.p, query_offsets, n_queries, mat, gap_open, gap_extend,
                 db->out_stage.p, s);
  if (rc != SW_OK) { (void)hipStreamSynchronize(s); return rc; }
  if (out_n > 0 && (e = hipMemcpyAsync(out_scores, db->out_stage.p, out_n * 4, hipMemcpyDeviceToHost,
                                       s)) != hipSuccess)
    return hip_fail(e, "score download");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
  set_error("");
  return SW_OK;
}

static int impl_set_option(swdb::Searcher* db, int32_t key, int64_t value) {
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
      if (value != 0 && value != 12 && value != 14 && value != 16 && value != 18 && value != 20 &&
          value != 32)
        return fail(SW_EINVAL, "rows must be 0, 12, 14, 16, 18, 20 or 32");
      db->opt_rows = (int32_t)value;
      return SW_OK;
    case SW_OPT_WAVES:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8 && value != 12 &&
          value != 16)
        return fail(SW_EINVAL, "waves must be 0, 1, 2, 4, 8, 12 or 16");
      db->opt_waves = (int32_t)value;
      return SW_OK;
    case SW_OPT_INTRA_ROWS:
      if (value != 0 && value != 2 && value != 4 && value != 8)
        return fail(SW_EINVAL, "intra rows must be 0, 2, 4 or 8");
      db->opt_intra_rows = (int32_t)value;
      return SW_OK;
    case SW_OPT_HYBRID_SHARE:
      if (value < 0 || value > 1000) return fail(SW_EINVAL, "hybrid share must be in 0..1000");
      db->hyb_share = (int32_t)value;
      return SW_OK;
    case SW_OPT_GRAPHS:
      if (value != 0 && value != 1) return fail(SW_EINVAL, "graphs must be 0 or 1");
      db->use_graphs = value != 0;
      db->batch.drop_graph();
      return SW_OK;
    case SW_OPT_INTRA_WAVES:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
        return fail(SW_EINVAL, "intra waves must be 0, 1, 2, 4 or 8");
      db->opt_intra_waves = (int32_t)value;
      return SW_OK;
    case SW_OPT_OFFLOAD_BINS:
      if (value < -1 || value > INT32_MAX)
        return fail(SW_EINVAL, "offloaded bins must be -1 (automatic) or 0..2^31-1");
      db->opt_offload = value;
      return SW_OK;
    default:
      return fail(SW_EINVAL, "unknown option " + std::to_string(key));
  }
}

static int impl_get_stats(swdb::Searcher* db, sw_stats* out) {
  using namespace swdb;
  if (!db || !out) return fail(SW_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
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
  if (db->flags.p && (db->d->plan.n_bins > 0 || db->d->plan.n_long > 0)) {
    if ((e = hipMemcpy(&cnt, db->flags.p, 4, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "stats");
  }
  st.n_rescored = cnt;
  *out = st;
  db->stats = sw_stats{};
  return SW_OK;
}

// ---------------------------------------------------------------- autotuner
// Candidate schedules: the inter-task (rows, waves) forms ((0, 0) = fitted to
// the query) and the long-pair kernel's (rows per lane, waves).
static const int kTuneR[SW_TUNE_CANDIDATES] = {0, 20, 18, 16, 14, 12, 14, 12};
static const int kTuneW[SW_TUNE_CANDIDATES] = {0, 12, 12, 12, 12, 12, 16, 16};
static const int kTuneIR[SW_TUNE_INTRA_CANDIDATES] = {2, 4, 8, 2, 4, 8, 2, 4, 8, 2, 4};
static const int kTuneIW[SW_TUNE_INTRA_CANDIDATES] = {1, 1, 1, 2, 2, 2, 4, 4, 4, 8, 8};

// Key of a tuning-cache entry: GPU architecture, compute units, a digest of
// the database's shape and the representative query lengths.
static std::string tune_key(const swdb::Searcher* db, const int (&rep_len)[SW_TUNE_BUCKETS]) {
  const swdb::DbData& d = *db->d;
  char arch[256] = "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d.device) == hipSuccess) {
    strncpy(arch, prop.gcnArchName, sizeof(arch) - 1);
    arch[sizeof(arch) - 1] = 0;
    for (char* c = arch; *c; ++c)
      if (*c == ' ' || *c == '\t') *c = '_';
  }
  // FNV-1a over the shape: counts, threshold and the log2-length histogram
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) { h ^= (v >> (8 * k)) & 0xffu; h *= 1099511628211ull; }
  };
  int64_t hist[32] = {};
  for (size_t i = 0; i + 1 < d.h_offs.size(); ++i) {
    const int64_t len = d.h_offs[i + 1] - d.h_offs[i];
    int lg = 0;
    while (lg < 31 && (int64_t(1) << lg) <= len) ++lg;
    ++hist[lg];
  }
  mix((uint64_t)d.n_seqs);
  mix((uint64_t)d.n_res);
  mix((uint64_t)d.plan.long_threshold);
  for (int64_t v : hist) mix((uint64_t)v);
  char buf[512];
  snprintf(buf, sizeof(buf), "%s cus=%d db=%016llx lens=%d,%d,%d,%d", arch, d.n_cus,
           (unsigned long long)h, rep_len[0], rep_len[1], rep_len[2], rep_len[3]);
  return buf;
}

// Sums the recorded kernel times of one kind and recycles the events.
static float drain_timed(swdb::Searcher* db, int kind) {
  float total = 0;
  for (auto& t : db->timed) {
    (void)hipEventSynchronize(t.b);
    float ms = 0;
    if (t.kind == kind && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) total += ms;
    db->ev_pool.push_back(t.a);
    db->ev_pool.push_back(t.b);
  }
  db->timed.clear();
  return total;
}

// Times each candidate schedule on this database with one random query (or
// query pair) of a representative length per bucket, and keeps the best per
// bucket; or applies a matching entry of the tuning cache.
static int impl_autotune(swdb::Searcher* db, const int32_t* query_lens, int32_t n_lens,
                         const char* cache_path, sw_tune_report* rep) {
  using namespace swdb;
  if (!db) return fail(SW_EINVAL, "db is NULL");
  if (n_lens < 0 || (n_lens > 0 && !query_lens)) return fail(SW_EINVAL, "bad query lengths");
  std::unique_lock<std::mutex> lk(db->mtx, std::try_to_lock);
  if (!lk.owns_lock()) return fail(SW_EBUSY, "another call is running on this handle");
  DeviceGuard g(db->d->device);
  sw_tune_report local{};
  for (int c = 0; c < SW_TUNE_CANDIDATES; ++c) {
    local.cand_rows[c] = kTuneR[c];
    local.cand_waves[c] = kTuneW[c];
  }
  for (int c = 0; c < SW_TUNE_INTRA_CANDIDATES; ++c) {
    local.intra_cand_rows[c] = kTuneIR[c];
    local.intra_cand_waves[c] = kTuneIW[c];
  }
  // representative lengths: the defaults, or the median of the caller's
  // lengths in each bucket (0: none there, the bucket stays untuned)
  int rep_len[SW_TUNE_BUCKETS] = {192, 448, 1280, 4096};
  if (n_lens > 0) {
    std::vector<int32_t> by[SW_TUNE_BUCKETS];
    for (int32_t i = 0; i < n_lens; ++i) {
      if (query_lens[i] < 0 || query_lens[i] > SW_MAX_LEN)
        return fail(SW_EINVAL, "query length out of range at " + std::to_string(i));
      if (query_lens[i] > 0) by[tune_bucket(query_lens[i])].push_back(query_lens[i]);
    }
    for (int b = 0; b < SW_TUNE_BUCKETS; ++b) {
      std::sort(by[b].begin(), by[b].end());
      rep_len[b] = by[b].empty() ? 0 : by[b][by[b].size() / 2];
    }
  }
  for (int b = 0; b < SW_TUNE_BUCKETS; ++b) local.query_len[b] = rep_len[b];
  auto apply = [&]() {
    for (int b = 0; b < SW_TUNE_BUCKETS; ++b) {
      db->tune_rows[b] = local.rows[b];
      db->tune_waves[b] = local.waves[b];
      db->tune_brows[b] = local.batch_rows[b];
      db->tune_bwaves[b] = local.batch_waves[b];
      db->tune_irows[b] = local.intra_rows[b];
      db->tune_iwaves[b] = local.intra_waves[b];
    }
  };
  const std::string key = cache_path ? tune_key(db, rep_len) : std::string();
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char line[1024];
      bool found = false;
      while (!found && fgets(line, sizeof(line), f)) {
        char* tab = strchr(line, '\t');
        if (!tab || std::string(line, tab) != key) continue;
        int v[6 * SW_TUNE_BUCKETS];
        int n = 0, off = 0, used = 0;
        const char* p = tab + 1;
        while (n < 6 * SW_TUNE_BUCKETS && sscanf(p + off, "%d%n", &v[n], &used) == 1) {
          off += used;
          ++n;
        }
        if (n != 6 * SW_TUNE_BUCKETS) continue;
        for (int b = 0; b < SW_TUNE_BUCKETS; ++b) {
          local.rows[b] = v[6 * b];
          local.waves[b] = v[6 * b + 1];
          local.batch_rows[b] = v[6 * b + 2];
          local.batch_waves[b] = v[6 * b + 3];
          local.intra_rows[b] = v[6 * b + 4];
          local.intra_waves[b] = v[6 * b + 5];
        }
        found = true;
      }
      fclose(f);
      if (found) {
        local.from_cache = 1;
        apply();
        if (rep) *rep = local;
        set_error("");
        return SW_OK;
      }
    }
  }
  if (db->d->n_seqs == 0 || db->d->plan.n_bins == 0) {
    if (rep) *rep = local;
    set_error("");
    return SW_OK;
  }
  Matrix mat{};
  // a BLOSUM-like synthetic matrix is enough to time the kernels: the cost
  // does not depend on the scores; +5 on the diagonal, -1 elsewhere
  for (int a = 0; a < SW_ALPHA; ++a)
    for (int b = 0; b < SW_ALPHA; ++b) mat.v[a * SW_ALPHA + b] = (int8_t)(a == b ? 5 : -1);
  int max_m = 1;
  for (int b = 0; b < SW_TUNE_BUCKETS; ++b) max_m = std::max(max_m, rep_len[b]);
  hipError_t e;
  hipStream_t s = db->own_stream;
  DevBuf<uint8_t> dq;
  DevBuf<int32_t> dout;
  dq.users = &db->users;
  dout.users = &db->users;
  struct Release {
    DevBuf<uint8_t>& a;
    DevBuf<int32_t>& b;
    ~Release() { a.release(); b.release(); }
  } release_guard{dq, dout};
  if ((e = dq.reserve((size_t)2 * max_m)) != hipSuccess ||
      (e = dout.reserve((size_t)2 * db->d->n_seqs)) != hipSuccess)
    return fail(SW_ENOMEM, std::string("autotune buffers: ") + hipGetErrorString(e));
  std::vector<uint8_t> hq((size_t)2 * max_m);
  uint32_t x = 12345u;
  for (auto& c : hq) { x = x * 1103515245u + 12345u; c = (uint8_t)((x >> 16) % 20); }
  if ((e = hipMemcpy(dq.p, hq.data(), hq.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "autotune upload");
  const bool saved_timing = db->timing, saved_graphs = db->use_graphs;
  const int32_t saved_r = db->opt_rows, saved_w = db->opt_waves;
  const int32_t saved_ir = db->opt_intra_rows, saved_iw = db->opt_intra_waves;
  const int64_t saved_off = db->opt_offload;
  db->timing = true;
  db->use_graphs = false;
  db->opt_offload = 0;   // the inter-task forms are measured over every bin
  int rc = SW_OK;
  // untuned while measuring, so the fitted candidate (0, 0) is what it says
  for (int b = 0; b < SW_TUNE_BUCKETS; ++b)
    db->tune_rows[b] = db->tune_waves[b] = db->tune_brows[b] = db->tune_bwaves[b] =
        db->tune_irows[b] = db->tune_iwaves[b] = 0;
  const bool has_long = db->d->plan.n_long > 0;
  for (int b = 0; b < SW_TUNE_BUCKETS && rc == SW_OK; ++b) {
    const int m = rep_len[b];
    if (m <= 0) continue;
    double best = -1, bbest = -1, ibest = 1e300;
    int pick = 0, bpick = 0, ipick = -1;
    db->opt_intra_rows = db->opt_intra_waves = 0;
    for (int c = 0; c < SW_TUNE_CANDIDATES && rc == SW_OK; ++c) {
      db->opt_rows = kTuneR[c];
      db->opt_waves = kTuneW[c];
      // single query: warm up, then two timed launches
      for (int rpt = 0; rpt < 3 && rc == SW_OK; ++rpt) {
        if (rpt == 1) { (void)drain_timed(db, kTimeInter); db->stats = sw_stats{}; }
        rc = enqueue_search(db, dq.p, m, mat, 10, 2, dout.p, s);
      }
      if (rc != SW_OK) break;
      float ms = drain_timed(db, kTimeInter);
      const double gc = ms > 0 ? (double)db->stats.inter_cells / (ms * 1e6) : 0;
      local.gcups[b][c] = (float)gc;
      if (gc > best) { best = gc; pick = c; }
      // batched: one pair of queries of this length
      const int64_t qo[3] = {0, m, 2 * (int64_t)m};
      db->stats = sw_stats{};
      for (int rpt = 0; rpt < 2 && rc == SW_OK; ++rpt) {
        if (rpt == 1) { (void)drain_timed(db, kTimeInter); db->stats = sw_stats{}; }
        rc = run_batch(db, dq.p, qo, 2, mat, 10, 2, dout.p, s);
      }
      if (rc != SW_OK) break;
      ms = drain_timed(db, kTimeInter);
      const double bgc = ms > 0 ? (double)db->stats.inter_cells / (ms * 1e6) : 0;
      local.batch_gcups[b][c] = (float)bgc;
      if (bgc > bbest) { bbest = bgc; bpick = c; }
    }
    // the long-pair kernel of single searches, beside the chosen inter-task
    // schedule
    db->opt_rows = kTuneR[pick];
    db->opt_waves = kTuneW[pick];
    for (int c = 0; has_long && c < SW_TUNE_INTRA_CANDIDATES && rc == SW_OK; ++c) {
      db->opt_intra_rows = kTuneIR[c];
      db->opt_intra_waves = kTuneIW[c];
      for (int rpt = 0; rpt < 2 && rc == SW_OK; ++rpt) {
        if (rpt == 1) (void)drain_timed(db, kTimeIntra);
        rc = enqueue_search(db, dq.p, m, mat, 10, 2, dout.p, s);
      }
      if (rc != SW_OK) break;
      const float ms = drain_timed(db, kTimeIntra);
      local.intra_ms[b][c] = ms;
      if (ms > 0 && ms < ibest) { ibest = ms; ipick = c; }
    }
    local.rows[b] = kTuneR[pick];
    local.waves[b] = kTuneW[pick];
    local.batch_rows[b] = kTuneR[bpick];
    local.batch_waves[b] = kTuneW[bpick];
    local.intra_rows[b] = ipick >= 0 ? kTuneIR[ipick] : 0;
    local.intra_waves[b] = ipick >= 0 ? kTuneIW[ipick] : 0;
  }
  (void)hipStreamSynchronize(s);
  (void)drain_timed(db, -1);
  db->batch.release();
  db->timing = saved_timing;
  db->use_graphs = saved_graphs;
  db->opt_rows = saved_r;
  db->opt_waves = saved_w;
  db->opt_intra_rows = saved_ir;
  db->opt_intra_waves = saved_iw;
  db->opt_offload = saved_off;
  db->stats = sw_stats{};
  if (rc != SW_OK) return rc;
  // (0, 0) chosen means "fitted": stored as untuned so the fit stays per query
  apply();
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (!f) return fail(SW_EINVAL, std::string("cannot write the tuning cache ") + cache_path);
    fprintf(f, "%s\t", key.c_str());
    for (int b = 0; b < SW_TUNE_BUCKETS; ++b)
      fprintf(f, "%d %d %d %d %d %d ", local.rows[b], local.waves[b], local.batch_rows[b],
              local.batch_waves[b], local.intra_rows[b], local.intra_waves[b]);
    fprintf(f, "\n");
    if (fclose(f) != 0)
      return fail(SW_EINVAL, std::string("cannot write the tuning cache ") + cache_path);
  }
  if (rep) *rep = local;
  set_error("");
  return SW_OK;
}

// ------------------------------------------------------------ public entry
// points: a database handle searches with its own searcher, a context with
// its private one.
static swdb::Searcher* S_of(sw_db* h) { return h ? &h->main : nullptr; }
static swdb::Searcher* S_of(sw_ctx* c) { return c ? &c->s : nullptr; }

int sw_search(sw_db* h, const uint8_t* query, int32_t query_len, const int8_t* matrix,
              int32_t gap_open, int32_t gap_extend, int32_t* out_scores) {
  return impl_search(S_of(h), query, query_len, matrix, gap_open, gap_extend, out_scores);
}
int sw_search_async(sw_db* h, const uint8_t* d_query, int32_t query_len, const int8_t* matrix,
                    int32_t gap_open, int32_t gap_extend, int32_t* d_out_scores, void* hip_stream) {
  return impl_search_async(S_of(h), d_query, query_len, matrix, gap_open, gap_extend, d_out_scores,
                           hip_stream);
}
int sw_search_async_noalloc(sw_db* h, const uint8_t* d_query, int32_t query_len,
                            const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                            int32_t* d_out_scores, void* hip_stream) {
  return impl_search_async_noalloc(S_of(h), d_query, query_len, matrix, gap_open, gap_extend,
                                   d_out_scores, hip_stream);
}
int sw_traceback(sw_db* h, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                 int32_t gap_open, int32_t gap_extend, const int32_t* seqs, int32_t n_items,
                 sw_alignment* out, uint32_t* ops, int64_t ops_cap, int64_t* ops_used) {
  return impl_traceback(S_of(h), query, query_len, matrix, gap_open, gap_extend, seqs, n_items,
                        out, ops, ops_cap, ops_used);
}

int sw_search_topk(sw_db* h, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                   int32_t gap_open, int32_t gap_extend, int32_t k, int32_t* out_scores,
                   sw_hit* out_hits) {
  return impl_search_topk(S_of(h), query, query_len, matrix, gap_open, gap_extend, k, out_scores,
                          out_hits);
}
int sw_search_topk_async(sw_db* h, const uint8_t* d_query, int32_t query_len,
                         const int8_t* matrix, int32_t gap_open, int32_t gap_extend, int32_t k,
                         int32_t* d_out_scores, sw_hit* d_hits, void* hip_stream) {
  return impl_search_topk_async(S_of(h), d_query, query_len, matrix, gap_open, gap_extend, k,
                                d_out_scores, d_hits, hip_stream);
}
int sw_search_hybrid(sw_db* h, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                     int32_t gap_open, int32_t gap_extend, int32_t cpu_threads,
                     int32_t* out_scores, sw_hybrid_stats* stats) {
  return impl_search_hybrid(S_of(h), query, query_len, matrix, gap_open, gap_extend, cpu_threads,
                            out_scores, stats);
}

int sw_host_search(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
                   const uint8_t* query, int32_t query_len, const int8_t* matrix,
                   int32_t gap_open, int32_t gap_extend, int32_t threads, int32_t* out_scores) {
  using namespace swdb;
  if (n_seqs < 0) return fail(SW_EINVAL, "n_seqs < 0");
  if (n_seqs > 0 && (!offsets || !out_scores)) return fail(SW_EINVAL, "offsets or out_scores is NULL");
  if (query_len < 0) return fail(SW_EINVAL, "query_len < 0");
  if (query_len > SW_MAX_LEN) return fail(SW_ERANGE, "query longer than 2^24-1 residues");
  if (query_len > 0 && !query) return fail(SW_EINVAL, "query is NULL");
  if (!matrix) return fail(SW_EINVAL, "matrix is NULL");
  if (gap_extend < 0 || gap_open < gap_extend)
    return fail(SW_EINVAL, "gaps must satisfy 0 <= gap_extend <= gap_open");
  if (gap_open > SW_MAX_GAP) return fail(SW_ERANGE, "gap_open > 2^30");
  if (threads < 0 || threads > 1024) return fail(SW_EINVAL, "threads must be 0..1024");
  if (n_seqs == 0) { set_error(""); return SW_OK; }
  if (offsets[0] != 0) return fail(SW_EINVAL, "offsets[0] must be 0");
  for (int64_t i = 0; i < n_seqs; ++i) {
    if (offsets[i + 1] < offsets[i]) return fail(SW_EINVAL, "offsets must be non-decreasing");
    if (offsets[i + 1] - offsets[i] > SW_MAX_LEN)
      return fail(SW_ERANGE, "sequence longer than 2^24-1 residues");
  }
  if (offsets[n_seqs] > 0 && !residues) return fail(SW_EINVAL, "residues is NULL");
  for (int64_t i = 0; i < offsets[n_seqs]; ++i)
    if (residues[i] >= SW_ALPHA) return fail(SW_EINVAL, "residue code >= 24");
  for (int32_t i = 0; i < query_len; ++i)
    if (query[i] >= SW_ALPHA) return fail(SW_EINVAL, "query code >= 24");
  cpu::Profile prof;
  try {
    cpu::build_profile(query, query_len, matrix, &prof);
  } catch (...) {
    return fail(SW_ENOMEM, "host allocation failed");
  }
  const int nt = threads > 0 ? threads : std::max(1, (int)std::thread::hardware_concurrency());
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    cpu::Workspace w;
    for (int64_t i; (i = next.fetch_add(1)) < n_seqs;) {
      const int64_t at = offsets[i];
      out_scores[i] = cpu::score(prof, residues + at, (int)(offsets[i + 1] - at), gap_open,
                                 gap_extend, &w);
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  } catch (...) {
  }
  worker();
  for (auto& t : pool) t.join();
  set_error("");
  return SW_OK;
}

int sw_search_mode(sw_db* h, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                   int32_t gap_open, int32_t gap_extend, int32_t mode, int32_t* out_scores) {
  return impl_search_mode(S_of(h), query, query_len, matrix, gap_open, gap_extend, mode,
                          out_scores);
}
int sw_search_mode_async(sw_db* h, const uint8_t* d_query, int32_t query_len,
                         const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                         int32_t mode, int32_t* d_out_scores, void* hip_stream) {
  return impl_search_mode_async(S_of(h), d_query, query_len, matrix, gap_open, gap_extend, mode,
                                d_out_scores, hip_stream);
}
int sw_search_batch(sw_db* h, const uint8_t* queries, const int64_t* query_offsets,
                    int32_t n_queries, const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                    int32_t* out_scores) {
  return impl_search_batch(S_of(h), queries, query_offsets, n_queries, matrix, gap_open,
                           gap_extend, out_scores);
}
int sw_search_batch_async(sw_db* h, const uint8_t* d_queries, const int64_t* query_offsets,
                          int32_t n_queries, const int8_t* matrix, int32_t gap_open,
                          int32_t gap_extend, int32_t* d_out_scores, void* hip_stream) {
  return impl_search_batch_async(S_of(h), d_queries, query_offsets, n_queries, matrix, gap_open,
                                 gap_extend, d_out_scores, hip_stream);
}
int sw_set_option(sw_db* h, int32_t key, int64_t value) {
  return impl_set_option(S_of(h), key, value);
}
int sw_get_stats(sw_db* h, sw_stats* out) { return impl_get_stats(S_of(h), out); }
int sw_autotune(sw_db* h, sw_tune_report* report) {
  return impl_autotune(S_of(h), nullptr, 0, nullptr, report);
}
int sw_autotune_ex(sw_db* h, const int32_t* query_lens, int32_t n_lens, const char* cache_path,
                   sw_tune_report* report) {
  return impl_autotune(S_of(h), query_lens, n_lens, cache_path, report);
}

int sw_ctx_create(sw_db* h, sw_ctx** out_ctx) {
  using namespace swdb;
  if (!out_ctx) return fail(SW_EINVAL, "out_ctx is NULL");
  *out_ctx = nullptr;
  if (!h) return fail(SW_EINVAL, "db is NULL");
  sw_ctx* c = new (std::nothrow) sw_ctx();
  if (!c) return fail(SW_ENOMEM, "host allocation failed");
  c->owner = h;
  DeviceGuard g(h->data.device);
  int rc = init_searcher(&c->s, &h->data);
  if (rc != SW_OK) {
    std::string msg = get_error();
    release_searcher(&c->s);
    delete c;
    set_error(msg);
    return rc;
  }
  {  // options start as the database handle's
    std::lock_guard<std::mutex> lk(h->main.mtx);
    c->s.timing = h->main.timing;
    c->s.use_graphs = h->main.use_graphs;
    c->s.sat_limit = h->main.sat_limit;
    c->s.opt_rows = h->main.opt_rows;
    c->s.opt_waves = h->main.opt_waves;
    c->s.opt_intra_rows = h->main.opt_intra_rows;
    c->s.opt_intra_waves = h->main.opt_intra_waves;
    c->s.opt_offload = h->main.opt_offload;
    for (int b = 0; b < SW_TUNE_BUCKETS; ++b) {
      c->s.tune_rows[b] = h->main.tune_rows[b];
      c->s.tune_waves[b] = h->main.tune_waves[b];
      c->s.tune_brows[b] = h->main.tune_brows[b];
      c->s.tune_bwaves[b] = h->main.tune_bwaves[b];
      c->s.tune_irows[b] = h->main.tune_irows[b];
      c->s.tune_iwaves[b] = h->main.tune_iwaves[b];
    }
  }
  *out_ctx = c;
  set_error("");
  return SW_OK;
}

void sw_ctx_free(sw_ctx* c) {
  if (!c) return;
  swdb::DeviceGuard g(c->owner->data.device);
  swdb::release_searcher(&c->s);
  delete c;
}

int64_t sw_ctx_bytes(const sw_db* h) {
  if (!h) return -1;
  const swdb::Plan& P = h->data.plan;
  return P.boundary_uint4 * 16 + (int64_t)swdb::kIntraGridRescore * swdb::rescore_stride(P) * 8 +
         (2 + 2 * std::max<int64_t>(P.n_bins * SW_BIN_SEQS + P.n_long, 1)) * 4 +
         std::max<int64_t>(h->data.n_seg_items, 1) * 4;
}

int sw_ctx_search_async(sw_ctx* c, const uint8_t* d_query, int32_t query_len,
                        const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                        int32_t* d_out_scores, void* hip_stream) {
  return impl_search_async(S_of(c), d_query, query_len, matrix, gap_open, gap_extend,
                           d_out_scores, hip_stream);
}
int sw_ctx_search_batch_async(sw_ctx* c, const uint8_t* d_queries, const int64_t* query_offsets,
                              int32_t n_queries, const int8_t* matrix, int32_t gap_open,
                              int32_t gap_extend, int32_t* d_out_scores, void* hip_stream) {
  return impl_search_batch_async(S_of(c), d_queries, query_offsets, n_queries, matrix, gap_open,
                                 gap_extend, d_out_scores, hip_stream);
}
int sw_ctx_set_option(sw_ctx* c, int32_t key, int64_t value) {
  return impl_set_option(S_of(c), key, value);
}
int sw_ctx_get_stats(sw_ctx* c, sw_stats* out) { return impl_get_stats(S_of(c), out); }

}  // extern "C"
