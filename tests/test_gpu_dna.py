"""GPU parity of DNA searches: nucleotide codes (A C G T N = 0..4) with a
match/mismatch table through the same C ABI and kernels as protein searches,
compared with the oracle score by score.  A planted copy of the query makes
some scores exceed the half-precision range (exact rescoring), and the long
sequences go through the intra-task kernel."""
import sys

import numpy as np
import pytest

import oracle.cpu as ocpu
import swinputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sw():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11100_amd as lib
    return lib


def _dna_db(seed, n=3000, plant=None):
    rng = np.random.default_rng(seed)
    lens = swinputs.lognormal_lengths(n, 1500.0, 0.8, 30, 12_000, rng)
    seqs = [swinputs.random_dna(int(L), rng) for L in lens]
    if plant is not None:
        for i in rng.choice(n, 4, replace=False):
            s = seqs[i]
            at = int(rng.integers(0, len(s) + 1))
            seqs[i] = np.concatenate([s[:at], plant, s[at:]])
    offs = np.zeros(n + 1, np.int64)
    np.cumsum([len(s) for s in seqs], out=offs[1:])
    return np.concatenate(seqs).astype(np.uint8), offs


@pytest.mark.parametrize("m,match,mismatch,go,ge", [(100, 5, 4, 10, 2), (1000, 5, 4, 16, 4),
                                                     (700, 1, 3, 5, 2), (3000, 2, 3, 5, 2)])
def test_dna_search_matches_oracle(sw, m, match, mismatch, go, ge):
    rng = np.random.default_rng(m)
    q = swinputs.random_dna(m, rng)
    q[rng.choice(m, max(1, m // 50), replace=False)] = 4      # a few N
    res, offs = _dna_db(m + 1, plant=q[: min(m, 900)])
    D = swinputs.dna_matrix(match, mismatch, -2)
    say("dna: m=%d, %d sequences, %d bases, +%d/-%d, gaps %d/%d"
        % (m, len(offs) - 1, offs[-1], match, mismatch, go, ge))
    with sw.Database(res, offs) as db:
        assert db.info()["n_long"] > 0
        got = db.search(q, D, go, ge)
        hits = db.search_topk(q, D, go, ge, k=8)
    want = ocpu.search(q, res, offs, D, go, ge)
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, [(int(i), int(got[i]), int(want[i])) for i in bad[:5]]
    assert want.max() > 2048 or match * min(m, 900) <= 2048
    order = ocpu.top_hits(want, 8)
    assert (hits["seq"] == order).all() and (hits["score"] == want[order]).all()
