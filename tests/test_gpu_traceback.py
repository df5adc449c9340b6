"""GPU parity of sw_traceback: the alignments of chosen database sequences
against the oracle's traceback (sw_gotoh_traceback) and, where the oracle's
Python tables would be too slow, against what is unique (score and end from
the C oracle) plus the alignment's own score from its definition
(alignment_score)."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import oracle.cpu as ocpu
import swinputs

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


def _check_valid(q, res, offs, al, S, go, ge):
    """The alignment lies in its sequence, scores what it says from the
    definition, and ends where it says."""
    sid = al["seq"]
    b = res[offs[sid]:offs[sid + 1]]
    if al["score"] == 0:
        assert al["ops"] == "" and al["query_begin"] == -1 and al["db_end"] == -1
        return
    sc, qe, de = oracle.alignment_score(q, b, S, go, ge, al["query_begin"], al["db_begin"],
                                        al["ops"])
    assert (sc, qe, de) == (al["score"], al["query_end"], al["db_end"]), al
    assert al["ops"][0] == "M" and al["ops"][-1] == "M"


@pytest.mark.parametrize("m,go,ge", [(1, 10, 2), (37, 10, 2), (150, 10, 2), (300, 5, 1),
                                     (130, 0, 0), (257, 11, 1), (90, 40, 1)])
def test_traceback_matches_oracle(sw, m, go, ge):
    """Every alignment equals the oracle's (begin, end, operations) on a
    ragged database (empty and one-residue sequences, lengths across pass
    and superstep boundaries), for every query shape the kernel's rows per
    lane take, and with the gap penalties that make ties common."""
    rng = np.random.default_rng(m + 7 * go + ge)
    lengths = np.concatenate([[0, 1, 2, 63, 64, 65, 127, 128, 129], rng.integers(3, 400, 40)])
    res, offs = swinputs.make_database(lengths.astype(np.int64), rng)
    q = swinputs.random_residues(m, rng)
    # a copy of part of the query with a deletion, inside one sequence
    big = int(np.argmax(lengths))
    res = res.copy()
    piece = np.delete(q[: min(m, 60)], min(m, 60) // 2) if m > 4 else q
    at = int(offs[big]) + 5
    res[at:at + len(piece)] = piece[: int(offs[big + 1]) - at]
    seqs = list(range(len(lengths))) + [big, 0]           # repeats allowed
    say("traceback m=%d gaps %d/%d" % (m, go, ge))
    with sw.Database(res, offs) as db:
        got = db.traceback(q, B62, go, ge, seqs)
    assert [g["seq"] for g in got] == seqs
    for al in got:
        sid = al["seq"]
        b = res[offs[sid]:offs[sid + 1]]
        want = oracle.sw_gotoh_traceback(q, b, B62, go, ge)
        assert (al["score"], al["query_begin"], al["db_begin"], al["query_end"], al["db_end"],
                al["ops"]) == want, (sid, al, want)
        _check_valid(q, res, offs, al, B62, go, ge)


def test_traceback_of_planted_copies_in_long_sequences(sw):
    """A 3,000-residue query copied into sequences of 9,000..20,000 residues
    (several passes of every kernel form and columns far past one segment):
    the alignment is the ungapped copy, begin and end at the copy."""
    rng = np.random.default_rng(21)
    q = swinputs.random_residues(3000, rng)
    lengths = np.array([9000, 20000, 12345, 500, 4000], np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    res = res.copy()
    places = {0: 100, 1: 15000, 2: 0}
    for sid, p in places.items():
        res[offs[sid] + p:offs[sid] + p + 3000] = q
    diag = int(sum(int(B62[c, c]) for c in q))
    with sw.Database(res, offs) as db:
        got = db.traceback(q, B62, 10, 2, [0, 1, 2, 3, 4])
    for al in got:
        sid = al["seq"]
        if sid in places:
            p = places[sid]
            assert (al["score"], al["query_begin"], al["db_begin"], al["query_end"],
                    al["db_end"], al["ops"]) == (diag, 0, p, 2999, p + 2999, "M" * 3000)
        _check_valid(q, res, offs, al, B62, 10, 2)
    for sid in (3, 4):
        b = res[offs[sid]:offs[sid + 1]]
        want = ocpu.score_end(q, b, B62, 10, 2)
        al = got[sid]
        assert (al["score"], al["query_end"], al["db_end"]) == want


def test_traceback_of_top_hits_full_size(sw):
    """The 10 best hits of the plain workload's longest query (5,478
    residues) against the 200,000-sequence database, whose codes span
    several 1 GiB groups: each alignment scores the hit's score from its
    definition and ends at the hit's end, both equal to the C oracle's."""
    w = swinputs.config("plain")
    q = w.queries[19]
    with sw.Database(w.residues, w.offsets) as db:
        hits = db.search_topk(q, w.matrix, 10, 2, k=10)
        got = db.traceback(q, w.matrix, 10, 2, hits["seq"])
    ids = hits["seq"].astype(np.int64)
    sc, qe, de = ocpu.search_end(q, w.residues, w.offsets, w.matrix, 10, 2, ids=ids)
    lens = np.diff(w.offsets)[ids]
    say("top-hit lengths", lens.tolist())
    for k, al in enumerate(got):
        assert al["seq"] == hits["seq"][k]
        assert (al["score"], al["query_end"], al["db_end"]) == (sc[k], qe[k], de[k])
        assert (al["score"], al["query_end"], al["db_end"]) == \
            (hits["score"][k], hits["query_end"][k], hits["db_end"][k])
        _check_valid(q, w.residues, w.offsets, al, w.matrix, 10, 2)


def test_traceback_arguments(sw):
    """Empty lists and queries, out-of-range sequences (SW_EINVAL), a too
    small operation buffer (SW_ERANGE with the size it needs, nothing
    written)."""
    rng = np.random.default_rng(5)
    res, offs = swinputs.make_database(rng.integers(10, 200, 30).astype(np.int64), rng)
    q = swinputs.random_residues(80, rng)
    L = sw._native.lib()
    m = np.ascontiguousarray(B62, dtype=np.int8)
    with sw.Database(res, offs) as db:
        assert db.traceback(q, B62, 10, 2, []) == []
        empty = db.traceback(np.zeros(0, np.uint8), B62, 10, 2, [3, 4])
        assert [(a["score"], a["ops"], a["db_begin"]) for a in empty] == [(0, "", -1)] * 2
        with pytest.raises(sw.SwError) as ei:
            db.traceback(q, B62, 10, 2, [30])
        assert ei.value.code == sw._native.SW_EINVAL
        with pytest.raises(sw.SwError) as ei:
            db.traceback(q, B62, 10, 2, [-1])
        assert ei.value.code == sw._native.SW_EINVAL
        ids = np.arange(30, dtype=np.int32)
        out = np.zeros(30, dtype=sw.ALIGNMENT_DTYPE)
        ops = np.full(4, 7, dtype=np.uint32)
        used = ctypes.c_int64()
        rc = L.sw_traceback(db._h, q.ctypes.data, len(q), m.ctypes.data, 10, 2,
                            ids.ctypes.data, 30, out.ctypes.data, ops.ctypes.data, 4,
                            ctypes.byref(used))
        assert rc == sw._native.SW_ERANGE and used.value > 4
        assert (ops == 7).all() and (out["n_ops"] == 0).all()
        full = db.traceback(q, B62, 10, 2, ids)
        assert sum(len(a["ops"]) > 0 for a in full) > 0
        n_runs = sum(len([1 for x in range(len(a["ops"])) if x == 0 or a["ops"][x] != a["ops"][x - 1]])
                     for a in full)
        assert n_runs == used.value
