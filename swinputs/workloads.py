"""Seeded synthetic workloads shaped like the paper's experiments.

The paper (section 4.1) searches 20 Swiss-Prot queries of lengths 144..5478
against UniProtKB/Swiss-Prot 2021_04 (565,928 sequences, 204,173,280 residues,
longest 35,213) with BLOSUM62 and gap penalties 10(2).  Neither the database
nor the queries are available here, so these generators draw stand-ins with
the same shape: log-normal database lengths, a 35,000-residue longest
sequence, i.i.d. residues from the background composition, and query lengths
spread geometrically over the same range.

Every generator takes an explicit seed; the same call gives the same bytes on
any machine.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from .background import BACKGROUND_FREQS
from .blosum62 import blosum62

GAP_OPEN = 10      # cost of a gap of length 1  ("10(2)", section 4.1)
GAP_EXTEND = 2     # cost of each further residue of the same gap

CONFIG_NAMES = ("plain-small", "plain", "batched", "long-mix", "served")

# stream tags keep independent draws independent of each other
_DB_LEN, _DB_RES, _QUERY, _EXTRA_Q, _ARRIVAL, _EMBED = 1, 2, 3, 4, 5, 6


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(tag)]))


def lognormal_lengths(n: int, mean: float, sigma: float, lo: int, hi: int,
                      rng: np.random.Generator) -> np.ndarray:
    """L = clip(rint(exp(N(mu, sigma^2))), lo, hi) with mu = ln(mean) - sigma^2/2."""
    mu = math.log(mean) - 0.5 * sigma * sigma
    raw = np.rint(np.exp(rng.normal(mu, sigma, size=n)))
    return np.clip(raw, lo, hi).astype(np.int64)


def random_residues(n: int, rng: np.random.Generator) -> np.ndarray:
    """n residue codes drawn i.i.d. from the background composition (codes 0..19)."""
    if n == 0:
        return np.zeros(0, dtype=np.uint8)
    # inverse-CDF sampling through a 2^16-entry table: code = LUT[u16]; each
    # residue's probability is its frequency rounded to a multiple of 2^-16
    cdf = np.cumsum(BACKGROUND_FREQS)
    cdf[-1] = 1.0
    lut = np.searchsorted(cdf, (np.arange(65536) + 0.5) / 65536.0, side="right")
    lut = lut.astype(np.uint8)
    u = rng.integers(0, 65536, size=n, dtype=np.uint16)
    return lut[u]


def make_database(lengths: np.ndarray, rng: np.random.Generator):
    """Concatenated residues (uint8[N]) and offsets (int64[n+1])."""
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    residues = random_residues(int(offsets[-1]), rng)
    return residues, offsets


def make_query(m: int, rng: np.random.Generator) -> np.ndarray:
    return random_residues(m, rng)


def geometric_query_lengths(k: int = 20, lo: int = 144, hi: int = 5478) -> List[int]:
    """round(lo * (hi/lo)^(i/(k-1))), i = 0..k-1: 144, 174, ..., 5478 for the defaults."""
    return [int(round(lo * (hi / lo) ** (i / (k - 1)))) for i in range(k)]


@dataclasses.dataclass
class Workload:
    name: str
    residues: np.ndarray           # uint8[N], codes < 24
    offsets: np.ndarray            # int64[n+1]
    queries: List[np.ndarray]      # uint8 arrays
    matrix: np.ndarray             # int8[24, 24], row = query code
    gap_open: int
    gap_extend: int
    arrivals: Optional[np.ndarray] = None   # seconds, for the served workload
    recipe: str = ""

    @property
    def n_seqs(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_residues(self) -> int:
        return int(self.offsets[-1])

    def seq(self, i: int) -> np.ndarray:
        return self.residues[self.offsets[i]:self.offsets[i + 1]]

    def cells(self) -> int:
        """Real DP cells m * N summed over the queries (the GCUPS numerator)."""
        return int(sum(len(q) for q in self.queries)) * self.n_residues


def _plain_db(seed: int, n: int = 200_000, mean: float = 355.0, max_len: int = 35_000):
    lens = lognormal_lengths(n, mean, 0.75, 20, max_len, _rng(seed, _DB_LEN))
    lens[int(np.argmax(lens))] = max_len
    return make_database(lens, _rng(seed, _DB_RES))


def config(name: str, seed: int = 0, *, scale: float = 1.0, qps: float = 50.0,
           n_requests: int = 2000) -> Workload:
    """Builds one named workload.

    scale < 1 shrinks the database (sequence count) for quick tests while
    keeping the recipe; scale = 1 is the full-size workload.
    """
    mat = blosum62()
    if name == "plain-small":
        lens = lognormal_lengths(2000, 350.0, 0.75, 20, 2000, _rng(seed, _DB_LEN))
        res, offs = make_database(lens, _rng(seed, _DB_RES))
        q = [make_query(144, _rng(seed, _QUERY))]
        return Workload(name, res, offs, q, mat, GAP_OPEN, GAP_EXTEND,
                        recipe="1 query (m=144) vs 2,000 log-normal sequences "
                               "(mean 350, sigma 0.75, clip 20..2000)")
    if name in ("plain", "batched", "served"):
        n = max(1, int(round(200_000 * scale)))
        res, offs = _plain_db(seed, n=n)
        qrng = _rng(seed, _QUERY)
        queries = [make_query(m, qrng) for m in geometric_query_lengths()]
        if name == "plain":
            return Workload(name, res, offs, queries, mat, GAP_OPEN, GAP_EXTEND,
                            recipe="20 queries (144..5478, geometric) vs %d log-normal "
                                   "sequences (mean 355, sigma 0.75, clip 20..35000, "
                                   "longest set to 35000)" % n)
        if name == "batched":
            xr = _rng(seed + 1, _EXTRA_Q)
            extra = xr.integers(50, 5001, size=200)
            queries = queries + [make_query(int(m), xr) for m in extra]
            return Workload(name, res, offs, queries, mat, GAP_OPEN, GAP_EXTEND,
                            recipe="the 20 plain queries + 200 queries of length "
                                   "U[50, 5000] against the plain database")
        # served
        arng = _rng(seed, _ARRIVAL)
        mlens = lognormal_lengths(n_requests, 400.0 * math.exp(0.5 * 0.8 ** 2), 0.8,
                                  30, 5000, arng)
        reqs = [make_query(int(m), arng) for m in mlens]
        gaps = arng.exponential(1.0 / qps, size=n_requests)
        return Workload(name, res, offs, reqs, mat, GAP_OPEN, GAP_EXTEND,
                        arrivals=np.cumsum(gaps),
                        recipe="%d requests, Poisson arrivals at %.1f QPS, lengths "
                               "log-normal (median 400, sigma 0.8, clip 30..5000)"
                               % (n_requests, qps))
    if name == "long-mix":
        n_short = max(1, int(round(49_000 * scale)))
        n_long = max(1, int(round(1_000 * scale)))
        lrng = _rng(seed, _DB_LEN)
        short = lognormal_lengths(n_short, 350.0, 0.75, 20, 9_999, lrng)
        long_ = lrng.integers(10_000, 35_001, size=n_long).astype(np.int64)
        lens = np.concatenate([short, long_])
        order = lrng.permutation(len(lens))
        lens = lens[order]
        res, offs = make_database(lens, _rng(seed, _DB_RES))
        qrng = _rng(seed, _QUERY)
        queries = [make_query(1000 * (k + 1), qrng) for k in range(10)]
        # plant exact copies of the longest query inside 5 long sequences so that
        # their scores exceed the 16-bit range
        erng = _rng(seed, _EMBED)
        long_ids = np.nonzero(lens >= 10_000)[0]
        planted = erng.choice(long_ids, size=min(5, len(long_ids)), replace=False)
        qlong = queries[-1]
        for sid in planted:
            start = int(offs[sid])
            room = int(lens[sid]) - len(qlong)
            at = int(erng.integers(0, room + 1))
            res[start + at:start + at + len(qlong)] = qlong
        w = Workload(name, res, offs, queries, mat, GAP_OPEN, GAP_EXTEND,
                     recipe="%d log-normal (mean 350, clip 20..9999) + %d U[10000, 35000] "
                            "sequences, 10 queries 1000..10000; 5 long sequences carry an "
                            "exact copy of the 10000-residue query" % (n_short, n_long))
        w.planted = np.sort(planted)
        return w
    raise ValueError("unknown workload %r" % name)
