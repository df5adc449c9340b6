/*
 * CPU oracle: Smith-Waterman local alignment scores with affine gaps.
 * TEST INFRASTRUCTURE ONLY - used by the test suite, the smoke check and the
 * benchmark's CPU baseline; the GPU library neither links nor calls it.
 *
 * Score (paper section 2.2; gaps "10(2)" of section 4.1 read as
 * w(k) = o + (k-1) e): Gotoh's recurrence over query rows i and database
 * columns j,
 *     E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o)
 *     F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)
 *     H(i,j) = max(0, H(i-1,j-1) + S(a_i, b_j), E(i,j), F(i,j))
 * with H = 0, E = F = -infinity on the borders; the score is max H.
 * Plain scalar code in 64-bit integers, one database sequence at a time;
 * POSIX threads take whole sequences from a shared counter.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define NEG_INF (INT64_MIN / 4)

static inline int64_t max2(int64_t x, int64_t y) { return x > y ? x : y; }

/* S is k x k, row = query code, column = database code. Returns -1 on
 * allocation failure. */
int64_t swo_score(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n,
                  const int8_t* S, int32_t k, int64_t o, int64_t e) {
  if (m == 0 || n == 0) return 0;
  int64_t* Hrow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* Frow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!Hrow || !Frow) { free(Hrow); free(Frow); return -1; }
  for (int64_t j = 0; j <= n; ++j) { Hrow[j] = 0; Frow[j] = NEG_INF; }
  int64_t best = 0;
  for (int64_t i = 1; i <= m; ++i) {
    const int8_t* Srow = S + (size_t)a[i - 1] * (size_t)k;
    int64_t h_diag = 0;      /* H(i-1, j-1) */
    int64_t h_left = 0;      /* H(i, j-1)   */
    int64_t E = NEG_INF;     /* E(i, j-1)   */
    for (int64_t j = 1; j <= n; ++j) {
      E = max2(E - e, h_left - o);
      Frow[j] = max2(Frow[j] - e, Hrow[j] - o);
      int64_t h = h_diag + Srow[b[j - 1]];
      h = max2(h, E);
      h = max2(h, Frow[j]);
      h = max2(h, 0);
      h_diag = Hrow[j];
      Hrow[j] = h;
      h_left = h;
      best = max2(best, h);
    }
  }
  free(Hrow);
  free(Frow);
  return best;
}

/* As swo_score, also returning the end of the best alignment: the cell
 * (i, j) with H(i, j) equal to the score that comes first in
 * database-then-query order (smallest j, then smallest i), as 0-based
 * residue indices *qend = i - 1, *dend = j - 1; (-1, -1) when the score is
 * 0.  Returns the score, or -1 on allocation failure. */
int64_t swo_score_end(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n,
                      const int8_t* S, int32_t k, int64_t o, int64_t e,
                      int64_t* qend, int64_t* dend) {
  *qend = *dend = -1;
  if (m == 0 || n == 0) return 0;
  int64_t* Hrow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* Frow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!Hrow || !Frow) { free(Hrow); free(Frow); return -1; }
  for (int64_t j = 0; j <= n; ++j) { Hrow[j] = 0; Frow[j] = NEG_INF; }
  int64_t best = 0, bi = 0, bj = 0;
  for (int64_t i = 1; i <= m; ++i) {
    const int8_t* Srow = S + (size_t)a[i - 1] * (size_t)k;
    int64_t h_diag = 0, h_left = 0, E = NEG_INF;
    for (int64_t j = 1; j <= n; ++j) {
      E = max2(E - e, h_left - o);
      Frow[j] = max2(Frow[j] - e, Hrow[j] - o);
      int64_t h = h_diag + Srow[b[j - 1]];
      h = max2(h, E);
      h = max2(h, Frow[j]);
      h = max2(h, 0);
      h_diag = Hrow[j];
      Hrow[j] = h;
      h_left = h;
      if (h > 0 && (h > best || (h == best && (j < bj || (j == bj && i < bi))))) {
        best = h;
        bi = i;
        bj = j;
      }
    }
  }
  free(Hrow);
  free(Frow);
  if (best > 0) { *qend = bi - 1; *dend = bj - 1; }
  return best;
}

/* Global (mode 1) and semi-global (mode 2) scores: Gotoh's recurrence
 * without the 0 in H's maximum, with borders H(i, 0) = -w(i) (the query's
 * leading residues), H(0, j) = -w(j) (global) or 0 (semi-global: free
 * leading database residues) and E(i, 0) = F(0, j) = -infinity; the score
 * is H(m, n) (global) or max_j H(m, j) (semi-global: free trailing database
 * residues), H(m, 0) when n = 0.  w(k) = o + (k - 1) e, w(0) = 0.  Returns
 * INT64_MIN on allocation failure. */
static int64_t gapw(int64_t k, int64_t o, int64_t e) { return k == 0 ? 0 : o + (k - 1) * e; }

int64_t swo_score_mode(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n,
                       const int8_t* S, int32_t k, int64_t o, int64_t e, int32_t mode) {
  if (n == 0) return -gapw(m, o, e);
  int64_t* Hrow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* Frow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!Hrow || !Frow) { free(Hrow); free(Frow); return INT64_MIN; }
  for (int64_t j = 0; j <= n; ++j) {   /* row 0 */
    Hrow[j] = mode == 1 ? -gapw(j, o, e) : 0;
    Frow[j] = NEG_INF;
  }
  for (int64_t i = 1; i <= m; ++i) {
    const int8_t* Srow = S + (size_t)a[i - 1] * (size_t)k;
    int64_t h_diag = Hrow[0];         /* H(i-1, 0) */
    int64_t h_left = -gapw(i, o, e);  /* H(i, 0) */
    int64_t E = NEG_INF;              /* E(i, 0) */
    Hrow[0] = h_left;
    for (int64_t j = 1; j <= n; ++j) {
      E = max2(E - e, h_left - o);
      Frow[j] = max2(Frow[j] - e, Hrow[j] - o);
      int64_t h = h_diag + Srow[b[j - 1]];
      h = max2(h, E);
      h = max2(h, Frow[j]);
      h_diag = Hrow[j];
      Hrow[j] = h;
      h_left = h;
    }
  }
  int64_t score = Hrow[n];
  if (mode != 1)
    for (int64_t j = 1; j <= n; ++j) score = max2(score, Hrow[j]);
  free(Hrow);
  free(Frow);
  return score;
}

typedef struct {
  const uint8_t* q; int64_t m;
  const uint8_t* res; const int64_t* offs;
  const int64_t* ids; int64_t n_items;
  const int8_t* S; int32_t k; int64_t o, e;
  int64_t* out;
  int64_t* qend;             /* with dend: ends wanted (swo_search_end) */
  int64_t* dend;
  int32_t mode;              /* 0 local, 1 global, 2 semi-global */
  int64_t next;
  int failed;
  pthread_mutex_t lock;
} job_t;

static void* worker(void* arg) {
  job_t* J = (job_t*)arg;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    int64_t it = J->next;
    J->next += 16;
    pthread_mutex_unlock(&J->lock);
    if (it >= J->n_items) break;
    int64_t end = it + 16 < J->n_items ? it + 16 : J->n_items;
    for (; it < end; ++it) {
      int64_t sid = J->ids ? J->ids[it] : it;
      int64_t b0 = J->offs[sid], n = J->offs[sid + 1] - b0;
      int64_t s;
      if (J->mode) {
        s = swo_score_mode(J->q, J->m, J->res + b0, n, J->S, J->k, J->o, J->e, J->mode);
        if (s == INT64_MIN) J->failed = 1;
      } else {
        s = J->qend ? swo_score_end(J->q, J->m, J->res + b0, n, J->S, J->k, J->o, J->e,
                                    &J->qend[it], &J->dend[it])
                    : swo_score(J->q, J->m, J->res + b0, n, J->S, J->k, J->o, J->e);
        if (s < 0) J->failed = 1;
      }
      J->out[it] = s;
    }
  }
  return NULL;
}

/* Scores of query q against database sequences ids[0..n_items) (all sequences
 * 0..n_items-1 when ids is NULL); out[t] is the score of item t.
 * Returns 0, or -1 on a thread or allocation failure. */
static int run_search(job_t* Jp, int32_t n_threads);

int swo_search(const uint8_t* q, int64_t m, const uint8_t* res, const int64_t* offs,
               const int64_t* ids, int64_t n_items, const int8_t* S, int32_t k,
               int64_t o, int64_t e, int64_t* out, int32_t n_threads) {
  job_t J = {q, m, res, offs, ids, n_items, S, k, o, e, out, NULL, NULL, 0, 0, 0,
             PTHREAD_MUTEX_INITIALIZER};
  return run_search(&J, n_threads);
}

/* swo_search for the global (mode 1) or semi-global (mode 2) score. */
int swo_search_mode(const uint8_t* q, int64_t m, const uint8_t* res, const int64_t* offs,
                    const int64_t* ids, int64_t n_items, const int8_t* S, int32_t k, int64_t o,
                    int64_t e, int32_t mode, int64_t* out, int32_t n_threads) {
  if (mode != 1 && mode != 2) return -1;
  job_t J = {q, m, res, offs, ids, n_items, S, k, o, e, out, NULL, NULL, mode, 0, 0,
             PTHREAD_MUTEX_INITIALIZER};
  return run_search(&J, n_threads);
}

/* swo_search with the ends of the best alignments (swo_score_end) in
 * qend[t], dend[t]. */
int swo_search_end(const uint8_t* q, int64_t m, const uint8_t* res, const int64_t* offs,
                   const int64_t* ids, int64_t n_items, const int8_t* S, int32_t k,
                   int64_t o, int64_t e, int64_t* out, int64_t* qend, int64_t* dend,
                   int32_t n_threads) {
  job_t J = {q, m, res, offs, ids, n_items, S, k, o, e, out, qend, dend, 0, 0, 0,
             PTHREAD_MUTEX_INITIALIZER};
  return run_search(&J, n_threads);
}

static int run_search(job_t* J, int32_t n_threads) {
  if (n_threads < 1) n_threads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return -1;
  int started = 0;
  for (int t = 0; t < n_threads; ++t) {
    if (pthread_create(&th[t], NULL, worker, J) != 0) break;
    ++started;
  }
  if (started == 0) worker(J);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
  return J->failed ? -1 : 0;
}
