/*
 * swdb.h - Smith-Waterman protein database search on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper section 2.2, "Smith-Waterman Algorithm", case (b):
 * database similarity search, one-to-many): for a protein query a = a_1..a_m
 * and every sequence b = b_1..b_n of a database, return the best local
 * alignment score
 *
 *     SW(a, b) = max(0, max over chains (i_1,j_1) < ... < (i_r,j_r) of
 *                   sum_t S(a_{i_t}, b_{j_t}) - sum of gap costs),
 *
 * where the residues skipped between two matched pairs form one gap in each
 * sequence and a gap of k >= 1 residues costs gap_open + (k-1) * gap_extend.
 * The paper's experiments (section 4.1) use BLOSUM62 and gap penalties
 * "10(2)", i.e. gap_open = 10, gap_extend = 2 under this convention; a caller
 * who reads "10(2)" as 10 + 2k passes gap_open = 12.
 *
 * Scores are exact 32-bit integers, identical to Gotoh's H/E/F recurrence
 * evaluated in unbounded integers.  Internally most cells are computed in
 * packed IEEE half precision, which is exact for integers up to 2048; any
 * sequence whose half-precision score reaches the rescoring limit (at most
 * 2048) is rescored exactly in 32-bit integer arithmetic.  Which kernel
 * scores a sequence depends on its length (paper section 2.3: inter-task or
 * intra-task parallelism depending on the sequence length):
 *  - shorter than `long_threshold`: the packed half-precision inter-task
 *    kernel (two sequences per lane);
 *  - single searches, at least `long_threshold`: an anti-diagonal wavefront
 *    (intra-task) kernel computing two such sequences at once in the two
 *    packed half-precision halves of every register, with the same exact
 *    rescoring;
 *  - batched searches: sequences below 4 x `long_threshold` go through the
 *    packed batched inter-task kernel (two queries per lane), longer ones
 *    through the 32-bit intra-task kernel.
 *
 * Conventions (all entry points):
 *  - Residue codes are bytes 0..23 in BLOSUM order
 *    A R N D C Q E G H I L K M F P S T W Y V B Z X *  (SW_ALPHA = 24).
 *  - The substitution matrix is int8_t[SW_ALPHA * SW_ALPHA], row-major,
 *    matrix[q * SW_ALPHA + t] = score of query residue q against database
 *    residue t.  It is a host pointer, read during the call only.
 *  - Nothing depends on the alphabet beyond the codes and the matrix: DNA
 *    (SW# aligns DNA as well as protein, paper section 2.3) uses codes 0..4
 *    for A C G T N and a match/mismatch table in the same calls.
 *  - Gap penalties: 0 <= gap_extend <= gap_open <= SW_MAX_GAP.  (With
 *    gap_open < gap_extend the recurrence and the definition above differ;
 *    such calls are rejected.)
 *  - Sizes: query and database sequences shorter than 2^24 residues; at most
 *    2^31 - 1 database sequences.  Empty queries and empty sequences are
 *    valid and score 0.
 *  - Ownership: every input buffer stays owned by the caller and is only read
 *    during the call (until the stream work completes, for the _async calls).
 *    Output buffers are caller-allocated.  A database handle owns its device
 *    memory until sw_db_free.
 *  - Errors: every function returns SW_OK or an SW_E* code and never throws
 *    or aborts; sw_last_error() describes the most recent failure on the
 *    calling thread.  On SW_EINVAL / SW_ERANGE nothing is written to the
 *    outputs and no work is enqueued.  SW_EDEVICE carries the HIP error
 *    string.
 *  - Concurrency: one call at a time per database handle; a concurrent call
 *    returns SW_EBUSY.  _async calls serialise on the caller's HIP stream.
 */
#ifndef SWDB_H_
#define SWDB_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_ALPHA 24
#define SW_MAX_GAP (1 << 30)
#define SW_MAX_LEN ((1 << 24) - 1)

enum sw_status {
  SW_OK = 0,
  SW_EINVAL = 1,   /* invalid argument: null pointer, bad code, bad offsets, gaps */
  SW_ERANGE = 2,   /* a size beyond the documented limits */
  SW_ENOMEM = 3,   /* device or host allocation failed */
  SW_EDEVICE = 4,  /* a HIP runtime or kernel error */
  SW_EBUSY = 5     /* another call is running on the same handle */
};

typedef struct sw_db sw_db;

/* ------------------------------------------------------------------ database
 * sw_db_load: copies a protein database to the current HIP device and lays it
 * out for search (length-sorted, 128 sequences per bin, position-major
 * interleaved residues - the coalesced layout the paper's 2-D sequence array
 * gives, section 3.2, figures "matrix_usm"/"matrix_read").
 *   residues : host, uint8_t[offsets[n_seqs]], codes < SW_ALPHA.
 *   offsets  : host, int64_t[n_seqs + 1], offsets[0] = 0, non-decreasing;
 *              sequence i is residues[offsets[i] .. offsets[i+1]).
 *   n_seqs   : number of sequences, >= 0.
 *   out_db   : receives the handle (NULL on failure).
 * sw_db_load_ex additionally sets long_threshold: sequences with at least
 * this many residues use the intra-task kernel (<= 0 selects the default,
 * SW_DEFAULT_LONG_THRESHOLD).
 */
#define SW_DEFAULT_LONG_THRESHOLD 2048
int sw_db_load(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
               sw_db** out_db);
int sw_db_load_ex(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
                  int32_t long_threshold, sw_db** out_db);

/* Releases the handle and all its device memory; NULL is a no-op. */
void sw_db_free(sw_db* db);

/* Database statistics; any output pointer may be NULL.  n_long is the
 * number of sequences at or above the long threshold (the intra-task
 * kernel's list). */
int sw_db_info(const sw_db* db, int64_t* n_seqs, int64_t* n_residues, int32_t* max_len,
               int64_t* n_long);

/* ------------------------------------------------------------------- search
 * sw_search: scores one query against every database sequence (synchronous,
 * host buffers).
 *   query      : host, uint8_t[query_len], codes < SW_ALPHA.
 *   out_scores : host, int32_t[n_seqs], in the database's original order.
 */
int sw_search(sw_db* db, const uint8_t* query, int32_t query_len, const int8_t* matrix,
              int32_t gap_open, int32_t gap_extend, int32_t* out_scores);

/* sw_search_async: as sw_search with device buffers, enqueued on hip_stream
 * (a hipStream_t; NULL = the null stream) and returning without waiting.
 *   d_query      : device, uint8_t[query_len].  Codes are not validated on
 *                  the device; codes >= SW_ALPHA give unspecified scores (but
 *                  never out-of-bounds accesses).
 *   d_out_scores : device, int32_t[n_seqs].
 * The handle's internal buffers are reused by the next call, so the caller
 * must not start another call on the handle from a different stream before
 * this one completes. */
int sw_search_async(sw_db* db, const uint8_t* d_query, int32_t query_len,
                    const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                    int32_t* d_out_scores, void* hip_stream);

/* sw_search_batch: many queries against the resident database in one
 * persistent launch: the same per-sequence scores as one sw_search per query
 * (paper section 4.1 searches 20 queries against one database; section 2.2,
 * case (b): every query against every database sequence, each pair an
 * independent alignment matrix).  Queries are sorted by length and paired, two queries
 * per 32-bit register lane; the work list of (query pair, half bin) items is
 * drained costliest first by a fixed grid of workgroups.  Repeating a batch
 * with the same query lengths, matrix, gaps and buffers replays a captured
 * HIP graph.
 *   queries       : host, concatenated codes, query q is
 *                   queries[query_offsets[q] .. query_offsets[q+1]).
 *   query_offsets : host, int64_t[n_queries + 1].
 *   out_scores    : host, int32_t[n_queries * n_seqs], row q = query q. */
int sw_search_batch(sw_db* db, const uint8_t* queries, const int64_t* query_offsets,
                    int32_t n_queries, const int8_t* matrix, int32_t gap_open,
                    int32_t gap_extend, int32_t* out_scores);

/* sw_search_batch_async: device queries/outputs, host query_offsets.
 *   d_queries    : device, uint8_t[query_offsets[n_queries]] (codes not
 *                  validated on the device, as for sw_search_async).
 *   d_out_scores : device, int32_t[n_queries * n_seqs].
 * The device buffers' sizes cannot be checked here; the caller guarantees
 * them (the Python binding checks them before the call). */
int sw_search_batch_async(sw_db* db, const uint8_t* d_queries, const int64_t* query_offsets,
                          int32_t n_queries, const int8_t* matrix, int32_t gap_open,
                          int32_t gap_extend, int32_t* d_out_scores, void* hip_stream);

/* sw_search_async_noalloc: sw_search_async for callers that cannot allocate
 * device memory - code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Same arguments, layouts and scores as
 * sw_search_async; it calls no hipMalloc, hipFree or other allocating
 * routine.  Its scratch is one array of SW_NOALLOC_SCRATCH_BYTES per GPU,
 * part of the library's code object: each GPU the library runs on holds it
 * until the process ends (its address is looked up and its boundary-row
 * part cleared when a database is first loaded on that GPU).  96 MiB of it
 * take the inter-task boundary rows of the short bins, launched in chunks
 * that fit (512 bytes per padded bin column); the rest takes the rescoring
 * list (8 bytes per sequence), the query's profiles (about 300 bytes per
 * query residue), and boundary rows of the long-sequence and rescoring
 * kernels (8 bytes per residue of the longest sequence per workgroup; their
 * grids shrink to what fits).  Calls that need more - a short bin longer
 * than 196,608 residues, or fixed parts plus one row of each intra-task
 * kernel beyond the array - return SW_ERANGE and enqueue nothing.
 * Every call on a GPU shares that GPU's array and leaves it in the state the
 * next call needs (zeros in the boundary-row part), so calls on one GPU must
 * not overlap: issue them on one stream, or order them with events; calls
 * that overlap on one GPU race and give wrong scores.  Timing (SW_OPT_TIMING)
 * is not recorded for these calls. */
#define SW_NOALLOC_SCRATCH_BYTES (128u << 20)
int sw_search_async_noalloc(sw_db* db, const uint8_t* d_query, int32_t query_len,
                            const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                            int32_t* d_out_scores, void* hip_stream);

/* ------------------------------------------------------------------ top hits
 * sw_search_topk: one search (as sw_search) followed by its k best hits with
 * the end of each hit's best local alignment.  A search tool reports the
 * best-scoring database sequences and their alignments, not only one value
 * per sequence (paper section 2.3, SW# "computes biological sequence
 * alignments"); the end cell is where the traceback of that alignment would
 * start.
 *   k          : 0 <= k <= SW_MAX_TOPK (SW_ERANGE above); min(k, n_seqs) hits
 *                are returned.
 *   out_scores : host, int32_t[n_seqs] (every score, as sw_search), or NULL.
 *   out_hits   : host, sw_hit[min(k, n_seqs)], best first: higher score
 *                first, equal scores by smaller sequence index.
 * A hit's end is the cell (query_end, db_end) holding its score that comes
 * first in database-then-query order (the smallest database position, then
 * the smallest query position), as 0-based residue indices; a score of 0
 * (no aligned pair scores above 0) has no end and reports (-1, -1).  The
 * selection runs on the device over the exact scores; the ends come from an
 * exact 32-bit pass over the k hit sequences only, so the search itself
 * costs the same as sw_search. */
#define SW_MAX_TOPK 4096
typedef struct sw_hit {
  int32_t seq;        /* database sequence index (original order) */
  int32_t score;      /* its score */
  int32_t query_end;  /* query position of the alignment's last pair, or -1 */
  int32_t db_end;     /* database-sequence position of that pair, or -1 */
} sw_hit;
int sw_search_topk(sw_db* db, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                   int32_t gap_open, int32_t gap_extend, int32_t k, int32_t* out_scores,
                   sw_hit* out_hits);
/* sw_search_topk_async: device query, score row and hit list (the score row
 * is required here: d_out_scores int32_t[n_seqs], d_hits sw_hit[min(k,
 * n_seqs)]), enqueued on hip_stream like sw_search_async. */
int sw_search_topk_async(sw_db* db, const uint8_t* d_query, int32_t query_len,
                         const int8_t* matrix, int32_t gap_open, int32_t gap_extend, int32_t k,
                         int32_t* d_out_scores, sw_hit* d_hits, void* hip_stream);

/* sw_traceback: the alignments themselves, for chosen database sequences
 * (a search's best hits): for each, an optimal local alignment of the query
 * with the sequence (paper section 2.3: SW# computes alignments, and a
 * search reports them for its best hits), ending at the end sw_search_topk
 * reports.  The exact 32-bit intra-task kernel recomputes each sequence's
 * matrix, keeping one traceback code per cell in device memory (query
 * length rounded up to 512 bytes per sequence residue; sequences go in
 * groups of up to 1 GiB of codes); the codes come back to the host, where
 * one thread per sequence walks back from the end.  Of several optimal
 * alignments it returns the one that, walking back, prefers a matched pair,
 * then a query residue against a gap, then a database residue against a
 * gap, and ends a gap at the first place it can.
 *   query, matrix : host, as sw_search.
 *   seqs      : host, n_items database sequence indices (any order,
 *               repeats allowed), 0 <= n_items <= SW_MAX_TOPK.
 *   out       : host, sw_alignment[n_items], in the order of seqs.
 *   ops       : host, uint32_t[ops_cap]: every alignment's operations in
 *               runs, (length << 2) | op with op 0 = M (a query residue
 *               against a database residue), 1 = I (a query residue against
 *               a gap), 2 = D (a database residue against a gap); alignment
 *               t's runs are ops[out[t].ops_offset .. + out[t].n_ops).  At
 *               most query_len + the sequence's length runs per alignment.
 *   ops_used  : host, or NULL: the runs all alignments take (also when
 *               ops_cap is too small: then SW_ERANGE and nothing written).
 * A score of 0 has no alignment: begins and ends -1, no runs.  A sequence
 * whose codes would exceed 4 GiB returns SW_ERANGE; codes that do not form
 * a path (a fault) return SW_EDEVICE.  Synchronous. */
typedef struct sw_alignment {
  int32_t seq;          /* database sequence index */
  int32_t score;        /* the alignment's score (the sequence's search score) */
  int32_t query_begin;  /* 0-based first and last query positions, or -1 */
  int32_t query_end;
  int32_t db_begin;     /* 0-based first and last database-sequence positions */
  int32_t db_end;
  int64_t ops_offset;   /* first run in ops */
  int32_t n_ops;        /* runs */
  int32_t reserved;
} sw_alignment;
int sw_traceback(sw_db* db, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                 int32_t gap_open, int32_t gap_extend, const int32_t* seqs, int32_t n_items,
                 sw_alignment* out, uint32_t* ops, int64_t ops_cap, int64_t* ops_used);

/* ---------------------------------------------------------- hybrid search
 * sw_search_hybrid: one query against every database sequence with host
 * cores and the GPU at once (paper section 2.3: SW#db uses CPUs and GPUs
 * simultaneously with dynamic work distribution; the experiments of section
 * 4.1 give the CPU side one thread, T=1).  The short bins' sequences form
 * one shared work order, longest first: the calling thread launches the
 * GPU's inter-task kernel on chunks of whole bins taken from the front (at
 * most two chunks queued, the next claimed when the earlier one ends),
 * while `cpu_threads` host threads (0: one fewer than the host's hardware
 * threads) take single sequences from the back and score them with the host
 * scorer (Farrar's striped 16-bit SIMD recurrence with exact 32-bit
 * rescoring, the code behind sw_host_search).  The split is planned from
 * both sides' rates measured by earlier calls on the handle: the GPU's first
 * chunk leaves the host twice its expected share, and a host thread gives
 * back a sequence it would not finish by the planned end, so the GPU never
 * waits long for the host; the bin where the two meet may be scored by
 * both (with identical scores).  Long sequences and the GPU's rescoring
 * stay on the GPU.  Scores are identical to sw_search.  Host buffers,
 * synchronous; `stats` may be NULL. */
typedef struct sw_hybrid_stats {
  int64_t gpu_bins;                /* short bins the GPU scored */
  int64_t cpu_seqs;                /* short sequences the host threads scored */
  int64_t gpu_cells, cpu_cells;    /* cells (query length x residues) of each side */
  int32_t cpu_threads;             /* host threads used */
  float ms;                        /* wall time of the call */
} sw_hybrid_stats;
int sw_search_hybrid(sw_db* db, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                     int32_t gap_open, int32_t gap_extend, int32_t cpu_threads,
                     int32_t* out_scores, sw_hybrid_stats* stats);

/* sw_host_search: the host scorer of the hybrid search on its own, over
 * host buffers laid out as for sw_db_load: every sequence's score against
 * the query, computed by `threads` host threads (0: all hardware threads).
 * It needs no GPU; the GPU entry points never call it. */
int sw_host_search(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
                   const uint8_t* query, int32_t query_len, const int8_t* matrix,
                   int32_t gap_open, int32_t gap_extend, int32_t threads, int32_t* out_scores);

/* ------------------------------------------------------------ other modes
 * sw_search_mode: one query against every database sequence with another
 * alignment operation of the same scoring scheme (paper section 2.3: SW#
 * aligns in several modes; section 5 names other alignment operations as
 * future work).  Every mode is a maximum over chains of matched pairs with
 * the local score's inner gap costs and no floor at 0:
 *   SW_MODE_LOCAL      : the local score (exactly sw_search);
 *   SW_MODE_GLOBAL     : the leading and trailing unmatched residues of each
 *                        sequence also form one gap each (Needleman-Wunsch
 *                        with affine gaps; an empty sequence scores
 *                        -w(query_len), w(k) = gap_open + (k-1) gap_extend,
 *                        w(0) = 0);
 *   SW_MODE_SEMIGLOBAL : the query is aligned end to end, the database
 *                        sequence's leading and trailing residues are free
 *                        (the query's best placement inside each sequence).
 * Scores are exact 32-bit integers and may be negative.  Calls whose scores
 * could leave +-2^28 - gap_open + (gap_extend + 128) x (query_len + 512 +
 * longest sequence + 1024) > 2^28 - return SW_ERANGE.  Sequences shorter
 * than the long threshold run in the int32 inter-task kernel (one sequence
 * per lane), longer ones in the int32 intra-task wavefront kernel.  Buffers
 * as sw_search / sw_search_async. */
enum sw_mode { SW_MODE_LOCAL = 0, SW_MODE_GLOBAL = 1, SW_MODE_SEMIGLOBAL = 2 };
int sw_search_mode(sw_db* db, const uint8_t* query, int32_t query_len, const int8_t* matrix,
                   int32_t gap_open, int32_t gap_extend, int32_t mode, int32_t* out_scores);
int sw_search_mode_async(sw_db* db, const uint8_t* d_query, int32_t query_len,
                         const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                         int32_t mode, int32_t* d_out_scores, void* hip_stream);

/* Description of the most recent failure on this thread ("" if none).  The
 * string stays valid until the next call on the same thread. */
const char* sw_last_error(void);

/* ------------------------------------------------------------ tuning, stats
 * sw_set_option: per-handle knobs.  Values outside the listed ranges return
 * SW_EINVAL.  */
enum sw_option {
  SW_OPT_TIMING = 1,      /* 0/1: record HIP events around every kernel */
  SW_OPT_SAT_LIMIT = 2,   /* 0..32767: a sequence whose half-precision score
                             reaches min(limit, 2048) is rescored in 32-bit
                             integers (default 32767, i.e. the whole exact
                             range; 0 rescores everything) */
  SW_OPT_ROWS = 3,        /* inter-task query rows per strip: 0 (auto: rows and
                             waves fitted to the query length from the
                             schedules' measured efficiencies), 12, 14, 16,
                             18, 20 (with 12 waves; 12 and 14 also with 16;
                             16 otherwise), 32 (not with 12 or 16 waves);
                             batched searches: 12 .. 20 with 12 waves, 12 and
                             14 with 16, 16 or 32 otherwise, auto fitted to
                             the pairs' lengths */
  SW_OPT_WAVES = 4,       /* inter-task waves per workgroup: 0 (auto), 1, 2, 4, 8, 12,
                             16 (12 not with 32 rows; 16 with 12 or 14 rows,
                             four waves per SIMD; batched searches: 4, 8, 12,
                             16) */
  SW_OPT_INTRA_ROWS = 5,  /* intra-task query rows per lane: 0 (auto), 2, 4, 8 */
  SW_OPT_INTRA_WAVES = 6, /* intra-task waves per long sequence: 0 (auto), 1, 2, 4, 8 */
  SW_OPT_HYBRID_SHARE = 8, /* hybrid search: 0 (default) plans the host's share
                             from measured rates; 1..1000 fixes it at that many
                             thousandths of the short bins' cells, with no
                             give-back (for tests and experiments) */
  SW_OPT_GRAPHS = 7,      /* 0/1: replay batched searches from a captured HIP graph
                             (default 1; graphs are not used while TIMING is on) */
  SW_OPT_OFFLOAD_BINS = 9  /* single searches (and top-k searches): how many of
                             the longest short bins (128 sequences each) the
                             long-pair kernel scores instead of the inter-task
                             kernel, two sequences per workgroup: -1 (default)
                             chooses per query, handing over bins while the
                             longest remaining one would outlast the whole
                             search on the device (queries long for the
                             database's size); 0 never; k >= 1 the k longest
                             (at most all).  Batched, hybrid and
                             allocation-free searches hand over none */
};
int sw_set_option(sw_db* db, int32_t key, int64_t value);

/* Counters accumulated over every query searched since the previous
 * sw_get_stats call (times are 0 for work enqueued with SW_OPT_TIMING off).
 * Kernel times come from HIP events recorded on the stream each kernel runs
 * on. */
typedef struct sw_stats {
  float ms_total;          /* first query's start to last query's end */
  float ms_inter;          /* inter-task kernel time, summed over launches */
  float ms_intra;          /* long-sequence intra-task kernel time, summed */
  float ms_rescore;        /* 32-bit rescoring kernel time, summed */
  int32_t n_inter_launches;
  int32_t n_rescored;      /* sequences rescored in 32 bits for the most
                              recent query */
  int64_t inter_cells;     /* real cells (query length x residues) given to
                              the inter-task kernel */
  int64_t intra_cells;     /* real cells given to the intra-task kernel */
  int32_t rows;            /* strip height of the last inter-task launch */
  int32_t waves;           /* waves per workgroup of the last inter-task launch */
  int32_t long_items;      /* work items of the last single search's long-list
                              kernel: pairs of long sequences, or (short
                              queries) column segments of those pairs */
  int32_t long_overlap;    /* columns each segment's window reaches back
                              (-1: the pairs were not cut into segments) */
} sw_stats;

/* Waits for the recorded work, fills *out and resets the counters. */
int sw_get_stats(sw_db* db, sw_stats* out);

/* sw_autotune: chooses the schedules of this database's searches by
 * measurement (the paper finds the GCUPS sensitive to the work-group size and
 * the best size different from SW#db's default, section 4.2).  Query lengths
 * fall in four buckets (m < 256, < 768, < 2048, longer); for each bucket it
 * searches one random query of a representative length and, with HIP events
 * around the kernels, times
 *  - every inter-task schedule (rows, waves) of the single-query kernel: the
 *    fitted choice (0, 0) and the seven forms 20/18/16/14/12 x 12 and
 *    14/12 x 16 (SW_TUNE_CANDIDATES), keeping the highest GCUPS;
 *  - the same schedules of the batched kernel on a pair of such queries;
 *  - every (rows per lane, waves) of the long-sequence kernel of single
 *    searches (SW_TUNE_INTRA_CANDIDATES, when the database has long
 *    sequences), keeping the shortest kernel time.
 * Later searches on the handle (and contexts created afterwards) use the
 * tuned entries of their query's bucket unless SW_OPT_ROWS / SW_OPT_WAVES /
 * SW_OPT_INTRA_ROWS / SW_OPT_INTRA_WAVES are set.  sw_autotune uses the
 * representative lengths 192, 448, 1280 and 4096 and takes a few seconds on
 * a 200,000-sequence database.  `report` may be NULL.  Errors leave the
 * handle untuned.
 *
 * sw_autotune_ex tunes for the caller's workload and can persist the result:
 *   query_lens : host, int32_t[n_lens], the lengths the caller will search
 *                (NULL / 0: the default lengths); a bucket's representative
 *                length is the median of the lengths in it, and buckets with
 *                none stay untuned (fitted schedules) - lengths that are all
 *                0 measure nothing and clear an earlier tuning;
 *   cache_path : NULL, or a text file of tuning results keyed by the GPU
 *                architecture name, its compute-unit count, a digest of the
 *                database's shape (sequence count, residues, long threshold,
 *                histogram of log2 lengths) and the representative lengths.
 *                A matching entry is applied without measuring (report
 *                from_cache = 1); otherwise the measured result is appended.
 *                An unreadable or unwritable file returns SW_EINVAL. */
#define SW_TUNE_BUCKETS 4
#define SW_TUNE_CANDIDATES 8
#define SW_TUNE_INTRA_CANDIDATES 11
typedef struct sw_tune_report {
  int32_t query_len[SW_TUNE_BUCKETS];            /* representative lengths (0: untuned) */
  int32_t cand_rows[SW_TUNE_CANDIDATES];         /* inter-task candidates ((0, 0) fitted) */
  int32_t cand_waves[SW_TUNE_CANDIDATES];
  float gcups[SW_TUNE_BUCKETS][SW_TUNE_CANDIDATES];        /* single-query kernel */
  float batch_gcups[SW_TUNE_BUCKETS][SW_TUNE_CANDIDATES];  /* batched kernel */
  int32_t rows[SW_TUNE_BUCKETS], waves[SW_TUNE_BUCKETS];   /* chosen */
  int32_t batch_rows[SW_TUNE_BUCKETS], batch_waves[SW_TUNE_BUCKETS];
  int32_t intra_cand_rows[SW_TUNE_INTRA_CANDIDATES];       /* long-sequence candidates */
  int32_t intra_cand_waves[SW_TUNE_INTRA_CANDIDATES];
  float intra_ms[SW_TUNE_BUCKETS][SW_TUNE_INTRA_CANDIDATES];  /* its kernel time, ms */
  int32_t intra_rows[SW_TUNE_BUCKETS], intra_waves[SW_TUNE_BUCKETS];  /* chosen (0: none) */
  int32_t from_cache;                            /* 1: applied from cache_path */
} sw_tune_report;
int sw_autotune(sw_db* db, sw_tune_report* report);
int sw_autotune_ex(sw_db* db, const int32_t* query_lens, int32_t n_lens, const char* cache_path,
                   sw_tune_report* report);

/* ----------------------------------------------------------- search contexts
 * A database handle carries one search context; sw_ctx_create adds more, each
 * with private scratch (boundary rows, profiles, rescoring list, batch plan),
 * streams and options, so that several searches of one resident database can
 * be in flight at once - one call at a time per context, any number of
 * contexts concurrently (the serving loop keeps one per in-flight request).
 * A context must be freed before its database.  Options start as the
 * database handle's at creation.
 *   sw_ctx_bytes : device bytes of fixed scratch one context allocates (per-
 *                  query buffers grow on top of it), or -1 for a NULL db. */
typedef struct sw_ctx sw_ctx;
int sw_ctx_create(sw_db* db, sw_ctx** out_ctx);
void sw_ctx_free(sw_ctx* ctx);
int64_t sw_ctx_bytes(const sw_db* db);
int sw_ctx_search_async(sw_ctx* ctx, const uint8_t* d_query, int32_t query_len,
                        const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                        int32_t* d_out_scores, void* hip_stream);
int sw_ctx_search_batch_async(sw_ctx* ctx, const uint8_t* d_queries,
                              const int64_t* query_offsets, int32_t n_queries,
                              const int8_t* matrix, int32_t gap_open, int32_t gap_extend,
                              int32_t* d_out_scores, void* hip_stream);
int sw_ctx_set_option(sw_ctx* ctx, int32_t key, int64_t value);
int sw_ctx_get_stats(sw_ctx* ctx, sw_stats* out);


/* ------------------------------------------------------- host-only layout
 * The database layout, computed without touching any device (the same code
 * sw_db_load uses).  Sequences are stable-sorted by decreasing length; those
 * with length >= long_threshold form the long list (scored by the intra-task
 * kernel in single searches); the rest fill the short bins of SW_BIN_SEQS =
 * 128 consecutive sorted sequences, slot k of a bin being lane k/2, half k%2.
 * The long sequences shorter than the very-long threshold (4 x long_threshold)
 * also fill "long bins", stored after the short bins, which batched searches
 * score with the inter-task kernel.  A bin stores its residues
 * position-major: dword res_off + (p/4)*128 + k holds positions p..p+3 of slot
 * k (byte p%4 = position p), padded with code SW_PAD_CODE up to the bin
 * length, a multiple of 4 and at least SW_MIN_BIN_LEN.  Each byte holds
 * 8 x the residue code (the byte offset of the code's dword pair in a
 * profile row pair).
 */
#define SW_BIN_SEQS 128
#define SW_PAD_CODE 24
#define SW_MIN_BIN_LEN 96

typedef struct sw_plan_info {
  int64_t n_bins;          /* bins of short sequences */
  int64_t n_long_bins;     /* bins of long sequences below the very-long threshold */
  int64_t n_long;          /* sequences in the long list */
  int64_t n_very_long;     /* long sequences at or above the very-long threshold */
  int64_t packed_dwords;   /* size of the interleaved residue store */
  int64_t boundary_bytes;  /* inter-task boundary-row scratch for all bins */
  int32_t max_len;         /* longest sequence */
  int32_t max_bin_len;     /* longest bin (padded) */
  int32_t max_long_len;    /* longest sequence in the long list (0 if none) */
  int32_t long_threshold;  /* the threshold actually used */
  int32_t very_long_threshold;
} sw_plan_info;

/* Validates offsets and fills *info.  residues may be NULL (codes are then
 * not checked). */
int sw_plan(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
            int32_t long_threshold, sw_plan_info* info);

/* Fills the host layout arrays sized from sw_plan (nb = n_bins + n_long_bins):
 *   packed   : uint32_t[packed_dwords]
 *   bin_desc : int64_t[nb * 4] = {res_off (dwords), boundary offset
 *              (16-byte units), length, first slot} per bin
 *   slot_seq : int32_t[nb * 128], original sequence index or -1
 *   long_ids : int32_t[n_long], original indices, longest first */
int sw_pack(const uint8_t* residues, const int64_t* offsets, int64_t n_seqs,
            int32_t long_threshold, uint32_t* packed, int64_t* bin_desc,
            int32_t* slot_seq, int32_t* long_ids);

#ifdef __cplusplus
}
#endif

#endif /* SWDB_H_ */
