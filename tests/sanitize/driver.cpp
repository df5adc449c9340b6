// Host code under AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure): the database layout (plan_layout / fill_layout) on
// random and edge-case databases, the hybrid search's host scorer against
// the C oracle on random inputs, and the oracle's own entry points.  Exits
// non-zero on the first mismatch; the sanitizers abort on any memory or
// undefined-behaviour error.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../../include/swdb.h"
#include "../../paper_2203_11100_amd/csrc/cpu_scorer.h"
#include "../../paper_2203_11100_amd/csrc/layout.h"
#include "../../paper_2203_11100_amd/csrc/trace_walk.h"

extern "C" {
int64_t swo_score(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const int8_t* S,
                  int32_t k, int64_t o, int64_t e);
int64_t swo_score_end(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const int8_t* S,
                      int32_t k, int64_t o, int64_t e, int64_t* qend, int64_t* dend);
int64_t swo_score_mode(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const int8_t* S,
                       int32_t k, int64_t o, int64_t e, int32_t mode);
int swo_search(const uint8_t* q, int64_t m, const uint8_t* res, const int64_t* offs,
               const int64_t* ids, int64_t n_items, const int8_t* S, int32_t k, int64_t o,
               int64_t e, int64_t* out, int32_t n_threads);
}

static int layout_case(std::mt19937& g, int n, int max_len, int t_long) {
  std::vector<int64_t> offs(n + 1, 0);
  for (int i = 0; i < n; ++i) offs[i + 1] = offs[i] + (int64_t)(g() % (max_len + 1));
  std::vector<uint8_t> res((size_t)offs[n] + 1);
  for (auto& r : res) r = (uint8_t)(g() % 24);
  swdb::Plan P;
  if (swdb::plan_layout(res.data(), offs.data(), n, t_long, &P) != SW_OK) return 1;
  const int64_t nb = P.n_bins + P.n_long_bins;
  std::vector<uint32_t> packed((size_t)P.packed_dwords + 1);
  std::vector<int64_t> bins((size_t)nb * 4 + 1);
  std::vector<int32_t> slots((size_t)nb * SW_BIN_SEQS + 1);
  std::vector<int32_t> longs((size_t)P.n_long + 1);
  swdb::fill_layout(res.data(), offs.data(), P, packed.data(), bins.data(), slots.data(),
                    longs.data());
  // every sequence is in exactly one bin slot or the long list
  std::vector<int> seen(n, 0);
  for (int64_t s = 0; s < P.n_bins * SW_BIN_SEQS; ++s)
    if (slots[(size_t)s] >= 0) ++seen[slots[(size_t)s]];
  for (int64_t t = 0; t < P.n_long; ++t) ++seen[longs[(size_t)t]];
  for (int i = 0; i < n; ++i)
    if (seen[i] != 1) return 2;
  return 0;
}

// Per-cell traceback codes of one local alignment problem, written here from
// the code definition (where H came from: 0, diagonal, F, E, the first equal
// in that order; bit 2: E of the next column opens; bit 3: F of the next row
// opens), with the first cell holding the maximum in (column, row) order.
// Then the library's walk, whose alignment must score that maximum (from
// the definition: S over matched pairs, o + (k-1) e per gap run) and end at
// that cell.
static int walk_case(std::mt19937& g) {
  const int k = 2 + (int)(g() % 4);
  const int m = (int)(g() % 40), n = (int)(g() % 60);
  std::vector<int> S((size_t)k * k);
  for (auto& x : S) x = (int)(g() % 9) - 4;
  std::vector<int> a((size_t)m), b((size_t)n);
  for (auto& x : a) x = (int)(g() % k);
  for (auto& x : b) x = (int)(g() % k);
  const int e = (int)(g() % 3), o = e + (int)(g() % 6);
  const int64_t ld = ((m + 7) / 8) * 8 + 8;
  std::vector<uint8_t> dir((size_t)(ld * (n + 1)), 0xff);
  const long NEG = -(1L << 40);
  std::vector<long> H((size_t)(m + 1) * (n + 1), 0), E(H.size(), NEG), F(H.size(), NEG);
  auto at = [&](int i, int j) { return (size_t)i * (n + 1) + j; };
  long best = 0;
  int bi = -1, bj = -1;
  for (int j = 1; j <= n; ++j)
    for (int i = 1; i <= m; ++i) {
      E[at(i, j)] = std::max(E[at(i, j - 1)] - e, H[at(i, j - 1)] - o);
      F[at(i, j)] = std::max(F[at(i - 1, j)] - e, H[at(i - 1, j)] - o);
      const long d = H[at(i - 1, j - 1)] + S[(size_t)a[i - 1] * k + b[j - 1]];
      const long h = std::max(std::max(0L, d), std::max(E[at(i, j)], F[at(i, j)]));
      H[at(i, j)] = h;
      const int src = h == 0 ? 0 : h == d ? 1 : h == F[at(i, j)] ? 3 : 2;
      const int eo = h - o >= E[at(i, j)] - e ? 4 : 0;
      const int fo = h - o >= F[at(i, j)] - e ? 8 : 0;
      dir[(size_t)((j - 1) * ld + (i - 1))] = (uint8_t)(src | eo | fo);
      if (h > best) { best = h; bi = i; bj = j; }
    }
  if (best == 0) return 0;
  int32_t qb = -1, db = -1;
  std::vector<uint32_t> runs;
  if (!swdb::walk_alignment(dir.data(), ld, bi - 1, bj - 1, &qb, &db, &runs)) return 1;
  long sc = 0;
  int i = qb, j = db;
  for (uint32_t r : runs) {
    const int len = (int)(r >> 2), op = (int)(r & 3);
    if (len < 1 || op > 2) return 2;
    if (op == 0) {
      for (int t = 0; t < len; ++t, ++i, ++j) {
        if (i >= m || j >= n) return 3;
        sc += S[(size_t)a[i] * k + b[j]];
      }
    } else {
      sc -= o + (long)(len - 1) * e;
      if (op == 1) i += len; else j += len;
    }
  }
  if (sc != best || i != bi || j != bj) return 4;
  return 0;
}

int main() {
  std::mt19937 g(12345);
  for (int c = 0; c < 2000; ++c)
    if (int r = walk_case(g)) { printf("traceback walk case %d: %d\n", c, r); return 1; }
  for (int c = 0; c < 60; ++c) {
    const int n = (int)(g() % 700);
    const int rc = layout_case(g, n, c % 3 == 0 ? 3000 : 400, c % 2 ? 0 : 250);
    if (rc) { printf("layout case %d failed (%d)\n", c, rc); return 1; }
  }
  int8_t S[24 * 24];
  for (int c = 0; c < 40; ++c) {
    for (auto& x : S) x = (int8_t)((int)(g() % 30) - 18);
    for (int i = 0; i < 24; ++i) S[i * 24 + i] = (int8_t)(1 + g() % 11);
    const int alpha = 2 + (int)(g() % 22);
    const int m = (int)(g() % 90), n = (int)(g() % 200);
    std::vector<uint8_t> a((size_t)m + 1), b((size_t)n + 1);
    for (auto& x : a) x = (uint8_t)(g() % alpha);
    for (auto& x : b) x = (uint8_t)(g() % alpha);
    const int e = (int)(g() % 4), o = e + (int)(g() % 12);
    swdb::cpu::Profile prof;
    swdb::cpu::build_profile(a.data(), m, S, &prof);
    swdb::cpu::Workspace w;
    const int64_t want = swo_score(a.data(), m, b.data(), n, S, 24, o, e);
    const int32_t got = swdb::cpu::score(prof, b.data(), n, o, e, &w);
    if (got != want) { printf("host scorer case %d: %d != %lld\n", c, got, (long long)want); return 1; }
    int64_t qe = 0, de = 0;
    if (swo_score_end(a.data(), m, b.data(), n, S, 24, o, e, &qe, &de) != want) return 1;
    for (int mode = 1; mode <= 2; ++mode) (void)swo_score_mode(a.data(), m, b.data(), n, S, 24, o, e, mode);
  }
  {
    std::vector<int64_t> offs = {0, 3, 3, 50, 120};
    std::vector<uint8_t> res(120), q(40);
    for (auto& x : res) x = (uint8_t)(g() % 20);
    for (auto& x : q) x = (uint8_t)(g() % 20);
    std::vector<int64_t> out(4);
    if (swo_search(q.data(), 40, res.data(), offs.data(), nullptr, 4, S, 24, 10, 2, out.data(), 3))
      return 1;
  }
  printf("ok\n");
  return 0;
}
