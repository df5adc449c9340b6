"""The allocation-free search (sw_search_async_noalloc) against the ordinary
device-buffer search (sw_search_async) on the same inputs, element by
element (scores are exact integers, so the bar is equality).

Two calls in a row on the library's one scratch array per GPU, the second
with a smaller input: first the full-size plain database (200,000 sequences,
whose inter-task boundary rows need several chunks of the scratch) with its
shortest query, then a small ragged database with long sequences and a
shorter query, plus forced rescoring of every sequence.  Every call goes
through the C ABI.
"""
import sys

import numpy as np
import pytest

import oracle.cpu as ocpu
import swinputs
from conftest import workload

pytestmark = pytest.mark.gpu

B62 = swinputs.blosum62()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sw():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11100_amd as lib
    return lib


def _both(sw, db, q, go=10, ge=2):
    """(ordinary, allocation-free) score rows of query q on one stream."""
    import torch
    dq = torch.from_numpy(np.ascontiguousarray(q, dtype=np.uint8)).cuda()
    a = torch.full((db.n_seqs,), -7, dtype=torch.int32, device="cuda")
    b = torch.full((db.n_seqs,), -7, dtype=torch.int32, device="cuda")
    db.search_async(dq, B62, go, ge, a)
    db.search_async_noalloc(dq, B62, go, ge, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def _small_db(seed):
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([[0, 1, 2, 33, 95, 96, 97], rng.integers(20, 700, 1500),
                              [2048, 2600, 3100, 5000, 9000]]).astype(np.int64)
    rng.shuffle(lengths)
    return swinputs.make_database(lengths, rng)


def test_noalloc_matches_search_async_twice(sw):
    w = workload("plain")
    info = sw.plan(w.offsets)
    assert info["boundary_bytes"] > 96 << 20      # several chunks of the scratch
    q = w.queries[0]
    say("noalloc: full-size plain database, m=%d" % len(q))
    with sw.Database(w.residues, w.offsets) as db:
        a, b = _both(sw, db, q)
    bad = np.nonzero(a != b)[0]
    assert len(bad) == 0, bad[:10]
    ids = np.random.default_rng(3).choice(len(a), 40, replace=False)
    assert (b[ids] == ocpu.search(q, w.residues, w.offsets, B62, 10, 2, ids=ids)).all()

    res, offs = _small_db(4)
    q2 = swinputs.random_residues(60, np.random.default_rng(5))
    say("noalloc: small ragged database with long sequences, m=60")
    with sw.Database(res, offs) as db:
        assert db.info()["n_long"] >= 5
        a, b = _both(sw, db, q2)
        assert (a == b).all(), np.nonzero(a != b)[0][:10]
        assert (b == ocpu.search(q2, res, offs, B62, 10, 2)).all()
        # every sequence through the exact rescoring kernel
        db.set_option(sw.SW_OPT_SAT_LIMIT, 0)
        a, b = _both(sw, db, q2)
        assert (a == b).all(), np.nonzero(a != b)[0][:10]
        assert (b == ocpu.search(q2, res, offs, B62, 10, 2)).all()


def test_noalloc_rejects_what_does_not_fit(sw):
    """A short bin whose boundary rows exceed the scratch's 96 MiB part (one
    200,000-residue sequence below a raised long threshold) is rejected with
    SW_ERANGE before anything is enqueued; the output stays untouched."""
    import torch
    rng = np.random.default_rng(6)
    res, offs = swinputs.make_database(np.array([200_000, 50, 70], np.int64), rng)
    q = torch.from_numpy(swinputs.random_residues(30, rng)).cuda()
    with sw.Database(res, offs, long_threshold=300_000) as db:
        out = torch.full((db.n_seqs,), -7, dtype=torch.int32, device="cuda")
        with pytest.raises(sw.SwError) as ei:
            db.search_async_noalloc(q, B62, 10, 2, out)
        assert ei.value.code == sw._native.SW_ERANGE
        torch.cuda.synchronize()
        assert (out.cpu().numpy() == -7).all()
