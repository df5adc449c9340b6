"""GPU parity of the global and semi-global modes (sw_search_mode).

Every score of every database sequence is compared with the C oracle's
swo_search_mode (Gotoh without the floor, borders per mode), element by
element; each call goes through the C ABI.
"""
import sys

import numpy as np
import pytest

import oracle.cpu as ocpu
import swinputs

pytestmark = pytest.mark.gpu

B62 = swinputs.blosum62()
MODES = ("global", "semiglobal")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sw():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11100_amd as lib
    return lib


def _ragged_db(seed=0, extra=(1500, 2100, 3000)):
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([
        [0, 0, 1, 2, 3, 4, 5, 7, 8, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257],
        rng.integers(20, 700, 1200), list(extra)]).astype(np.int64)
    rng.shuffle(lengths)
    return swinputs.make_database(lengths, rng)


def _check(got, q, res, offs, S, go, ge, mode):
    want = ocpu.search_mode(q, res, offs, S, go, ge, mode)
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, (mode, len(q), bad[:5], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("m", [1, 2, 15, 16, 17, 31, 32, 33, 100, 144, 600, 1300])
def test_modes_ragged_database(sw, mode, m):
    res, offs = _ragged_db()
    q = swinputs.random_residues(m, np.random.default_rng(100 + m))
    say("%s, m=%d" % (mode, m))
    with sw.Database(res, offs) as db:
        got = db.search_mode(q, B62, 10, 2, mode)
    _check(got, q, res, offs, B62, 10, 2, mode)


@pytest.mark.parametrize("gaps", [(0, 0), (5, 5), (11, 1), (40, 3), (1000, 1000)])
def test_modes_gap_penalties(sw, gaps):
    res, offs = _ragged_db(3)
    q = swinputs.random_residues(250, np.random.default_rng(7))
    go, ge = gaps
    with sw.Database(res, offs) as db:
        for mode in MODES:
            say("%s gaps %d/%d" % (mode, go, ge))
            _check(db.search_mode(q, B62, go, ge, mode), q, res, offs, B62, go, ge, mode)


def test_modes_long_list_every_schedule(sw):
    """The wavefront kernel's global/semi-global variants over long sequences,
    for every rows-per-lane and waves option and a query of several passes."""
    res, offs = _ragged_db(5)
    q = swinputs.random_residues(1100, np.random.default_rng(9))
    want = {md: ocpu.search_mode(q, res, offs, B62, 10, 2, md) for md in MODES}
    with sw.Database(res, offs, long_threshold=200) as db:
        for rr in (2, 4, 8):
            for w2 in (1, 2, 4, 8):
                db.set_option(sw.SW_OPT_INTRA_ROWS, rr)
                db.set_option(sw.SW_OPT_INTRA_WAVES, w2)
                for md in MODES:
                    say("long list %s rows=%d waves=%d" % (md, rr, w2))
                    got = db.search_mode(q, B62, 10, 2, md)
                    assert (got == want[md]).all(), (md, rr, w2)


def test_modes_closed_forms_and_empty(sw):
    """Self alignment and embedded copies (closed forms of the oracle's pins),
    an empty query and empty sequences, and the local mode equal to sw_search."""
    rng = np.random.default_rng(11)
    q = swinputs.random_residues(300, rng)
    diag = int(sum(int(B62[c, c]) for c in q))
    seqs = [q, np.concatenate([swinputs.random_residues(50, rng), q,
                               swinputs.random_residues(70, rng)]),
            np.zeros(0, np.uint8)] + [swinputs.random_residues(int(n), rng)
                                      for n in rng.integers(1, 400, 300)]
    offs = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(s) for s in seqs], out=offs[1:])
    res = np.concatenate(seqs)
    w = lambda k: 0 if k == 0 else 10 + 2 * (k - 1)
    with sw.Database(res, offs) as db:
        g = db.search_mode(q, B62, 10, 2, "global")
        s = db.search_mode(q, B62, 10, 2, "semiglobal")
        assert g[0] == diag and s[0] == diag and s[1] == diag
        assert g[2] == -w(len(q)) and s[2] == -w(len(q))
        _check(g, q, res, offs, B62, 10, 2, "global")
        _check(s, q, res, offs, B62, 10, 2, "semiglobal")
        e = np.zeros(0, np.uint8)
        assert (db.search_mode(e, B62, 10, 2, "global") == -np.array([w(len(x)) for x in seqs])).all()
        assert (db.search_mode(e, B62, 10, 2, "semiglobal") == 0).all()
        assert (db.search_mode(q, B62, 10, 2, "local") == db.search(q, B62, 10, 2)).all()
        with pytest.raises(sw.SwError):
            db.search_mode(q, B62, 1 << 27, 1 << 20, "global")     # beyond the 32-bit range


def test_modes_full_size_plain_database(sw):
    """Global and semi-global rows of the shortest plain query against the
    full 200,000-sequence database (every score compared)."""
    from conftest import workload
    w = workload("plain")
    q = w.queries[0]
    with sw.Database(w.residues, w.offsets) as db:
        for md in MODES:
            say("full plain database, %s, m=%d" % (md, len(q)))
            got = db.search_mode(q, w.matrix, 10, 2, md)
            _check(got, q, w.residues, w.offsets, w.matrix, 10, 2, md)
