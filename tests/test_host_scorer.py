"""The hybrid search's host scorer (sw_host_search, CPU only) against the
oracle: every score equal, on random and adversarial inputs - matrices with
all-negative rows and heavy mismatch penalties over 2..5-letter alphabets
(long vertical gaps that the lazy-F correction must carry across lanes;
stopping the correction one pass or one unit early fails these), gaps from
0 to beyond 16 bits, queries of every segment count, and scores beyond 16
bits (the 32-bit rescoring)."""
import numpy as np
import pytest

import oracle.cpu as ocpu
import swinputs

B62 = swinputs.blosum62()


@pytest.fixture(scope="module")
def sw():
    import paper_2203_11100_amd as lib
    return lib


def _db(seed, n=300, lo=0, hi=400):
    rng = np.random.default_rng(seed)
    lengths = rng.integers(lo, hi, n).astype(np.int64)
    return swinputs.make_database(lengths, rng)


@pytest.mark.parametrize("m", [1, 2, 15, 16, 17, 31, 32, 33, 100, 257, 700])
def test_host_scorer_blosum(sw, m):
    res, offs = _db(m)
    q = swinputs.random_residues(m, np.random.default_rng(1000 + m))
    got = sw.host_search(res, offs, q, B62, 10, 2, threads=4)
    assert (got == ocpu.search(q, res, offs, B62, 10, 2)).all()


@pytest.mark.parametrize("seed", range(6))
def test_host_scorer_adversarial_matrices(sw, seed):
    rng = np.random.default_rng(seed)
    S = rng.integers(-40, 12, (24, 24)).astype(np.int8)
    S[rng.integers(0, 24, 3)] = -60               # all-negative rows
    np.fill_diagonal(S, rng.integers(1, 15, 24))
    alpha = rng.integers(2, 6)
    lengths = rng.integers(0, 120, 200).astype(np.int64)
    offs = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=offs[1:])
    res = rng.integers(0, alpha, int(offs[-1])).astype(np.uint8)
    for m in (3, 16, 45, 130):
        q = rng.integers(0, alpha, m).astype(np.uint8)
        for go, ge in ((0, 0), (1, 1), (3, 1), (6, 6), (12, 2), (40, 1)):
            got = sw.host_search(res, offs, q, S, go, ge, threads=2)
            want = ocpu.search(q, res, offs, S, go, ge)
            assert (got == want).all(), (seed, m, go, ge, np.nonzero(got != want)[0][:5])


def test_host_scorer_large_gaps_and_scores(sw):
    rng = np.random.default_rng(7)
    q = swinputs.random_residues(3100, rng)
    W = 17
    seqs = [np.full(3500, W, np.uint8), q.copy(), swinputs.random_residues(500, rng),
            np.concatenate([swinputs.random_residues(40, rng), q])]
    offs = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(x) for x in seqs], out=offs[1:])
    res = np.concatenate(seqs)
    qw = np.full(3200, W, np.uint8)                       # W vs W: 11 x 3200 > 32767
    for query in (q, qw):
        for go, ge in ((10, 2), (40000, 40000), (1 << 30, 5)):
            got = sw.host_search(res, offs, query, B62, go, ge)
            assert (got == ocpu.search(query, res, offs, B62, go, ge)).all(), (go, ge)
    assert sw.host_search(res, offs, qw, B62, 10, 2)[0] == 11 * 3200


def test_host_scorer_rejects_bad_input(sw):
    res, offs = _db(1, n=5)
    q = np.zeros(5, np.uint8)
    with pytest.raises(sw.SwError):
        sw.host_search(res, offs, q, B62, 2, 3)           # open < extend
    bad = res.copy()
    bad[0] = 24
    with pytest.raises(sw.SwError):
        sw.host_search(bad, offs, q, B62, 10, 2)
    assert (sw.host_search(res, offs, np.zeros(0, np.uint8), B62, 10, 2) == 0).all()
