"""GPU parity of the top-k hits and their alignment ends (sw_search_topk).

The hit list is compared field by field with the oracle: the sequences are
the oracle's k best scores (higher first, equal scores by smaller index), and
each hit's score and (query end, database end) equal oracle.cpu.search_end
for that sequence (the first cell holding the score in database-then-query
order).  Every call goes through the C ABI.
"""
import sys

import numpy as np
import pytest

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


def _ragged_db(seed, n=1200, extra=(1500, 2100)):
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([[0, 0, 1, 2, 3, 31, 32, 33, 64, 65, 127, 128, 129],
                              rng.integers(20, 700, n), list(extra)]).astype(np.int64)
    rng.shuffle(lengths)
    return swinputs.make_database(lengths, rng)


def _check_hits(hits, scores, q, res, offs, S, go, ge, k):
    want_scores = ocpu.search(q, res, offs, S, go, ge)
    if scores is not None:
        assert (scores == want_scores).all(), np.nonzero(scores != want_scores)[0][:5]
    order = ocpu.top_hits(want_scores, k)
    assert len(hits) == len(order)
    assert (hits["seq"] == order).all(), (hits["seq"][:10], order[:10])
    s, qe, de = ocpu.search_end(q, res, offs, S, go, ge, ids=order)
    assert (hits["score"] == s).all()
    bad = np.nonzero((hits["query_end"] != qe) | (hits["db_end"] != de))[0]
    assert len(bad) == 0, [(int(order[i]), int(s[i]), (int(hits["query_end"][i]),
                            int(hits["db_end"][i])), (int(qe[i]), int(de[i]))) for i in bad[:5]]


@pytest.mark.parametrize("m,k", [(1, 5), (33, 1), (144, 100), (600, 257), (1300, 1000),
                                 (150, 4096)])
def test_topk_hits_match_oracle(sw, m, k):
    res, offs = _ragged_db(50)
    q = swinputs.random_residues(m, np.random.default_rng(51 + m))
    say("top-k m=%d k=%d" % (m, k))
    with sw.Database(res, offs) as db:
        hits, scores = db.search_topk(q, B62, 10, 2, k=k, scores=True)
    _check_hits(hits, scores, q, res, offs, B62, 10, 2, k)


def test_topk_ties_and_zero_scores(sw):
    """Many equal scores and equal maxima inside one matrix: duplicate
    sequences (equal scores, ranked by index), periodic sequences (the same
    maximum at several cells), and k beyond the positive scores (the rest of
    the list is score 0 with no end, by index)."""
    rng = np.random.default_rng(60)
    W, A, G = 17, 0, 7
    base = swinputs.random_residues(40, rng)
    seqs = [base.copy() for _ in range(30)]                       # equal scores
    seqs += [np.array([W, A] * r, np.uint8) for r in range(1, 40)]  # periodic
    seqs += [np.array([G] * r, np.uint8) for r in range(1, 20)]
    seqs += [np.zeros(0, np.uint8)] * 5
    seqs += [swinputs.random_residues(int(n), rng) for n in rng.integers(1, 300, 200)]
    order = rng.permutation(len(seqs))
    seqs = [seqs[i] for i in order]
    offs = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(s) for s in seqs], out=offs[1:])
    res = np.concatenate(seqs)
    queries = [np.array([W, A, W, A, W], np.uint8), base[5:25], np.array([G, G, G], np.uint8),
               np.array([W], np.uint8)]
    with sw.Database(res, offs) as db:
        for q in queries:
            for go, ge in ((10, 2), (0, 0), (3, 3)):
                say("ties: m=%d gaps %d/%d" % (len(q), go, ge))
                hits, scores = db.search_topk(q, B62, go, ge, k=len(seqs), scores=True)
                _check_hits(hits, scores, q, res, offs, B62, go, ge, len(seqs))


def test_topk_long_sequences_and_multipass_query(sw):
    """Hits among long sequences (the intra-task list) and a query of several
    passes; embedded copies of the query end at the copy's last residue."""
    rng = np.random.default_rng(70)
    q = swinputs.random_residues(1400, rng)
    lengths = np.concatenate([rng.integers(20, 600, 400), [2500, 3000, 5000, 9000]])
    res, offs = swinputs.make_database(lengths.astype(np.int64), rng)
    res = res.copy()
    # plant the query inside three sequences (two long)
    n = len(lengths)
    for sid, at in ((n - 1, 1234), (n - 3, 700), (5, None)):
        if at is None:
            at = 0
            ln = int(offs[sid + 1] - offs[sid])
            piece = q[:ln]
        else:
            piece = q
        res[offs[sid] + at: offs[sid] + at + len(piece)] = piece
    with sw.Database(res, offs) as db:
        say("long hits")
        hits, scores = db.search_topk(q, B62, 10, 2, k=20, scores=True)
    _check_hits(hits, scores, q, res, offs, B62, 10, 2, 20)
    # both full copies score the sum of the query's diagonal entries (a tie,
    # ranked by index) and end at the copy's last residue
    diag = int(sum(int(B62[c, c]) for c in q))
    assert list(hits["seq"][:2]) == [n - 3, n - 1] and (hits["score"][:2] == diag).all()
    assert (hits["query_end"][:2] == len(q) - 1).all()
    assert list(hits["db_end"][:2]) == [700 + len(q) - 1, 1234 + len(q) - 1]


def test_topk_empty_query_and_small_k(sw):
    res, offs = _ragged_db(80, n=100)
    with sw.Database(res, offs) as db:
        hits = db.search_topk(np.zeros(0, np.uint8), B62, 10, 2, k=7)
        assert (hits["seq"] == np.arange(7)).all() and (hits["score"] == 0).all()
        assert (hits["query_end"] == -1).all() and (hits["db_end"] == -1).all()
        assert len(db.search_topk(swinputs.random_residues(50, np.random.default_rng(1)),
                                  B62, 10, 2, k=0)) == 0
        with pytest.raises(sw.SwError):
            db.search_topk(np.zeros(5, np.uint8), B62, 10, 2, k=sw.SW_MAX_TOPK + 1)


def test_topk_async_on_device_buffers(sw):
    import torch
    res, offs = _ragged_db(90)
    q = swinputs.random_residues(300, np.random.default_rng(91))
    k = 64
    with sw.Database(res, offs) as db:
        d_out = torch.full((db.n_seqs,), -1, dtype=torch.int32, device="cuda")
        d_hits = torch.full((k, 4), -7, dtype=torch.int32, device="cuda")
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            db.search_topk_async(torch.from_numpy(q).cuda(), B62, 11, 1, k, d_out, d_hits,
                                 stream=stream)
        stream.synchronize()
        flat = d_hits.cpu().numpy()
    hits = np.zeros(k, dtype=sw.HIT_DTYPE)
    for i, name in enumerate(("seq", "score", "query_end", "db_end")):
        hits[name] = flat[:, i]
    _check_hits(hits, d_out.cpu().numpy(), q, res, offs, B62, 11, 1, k)


def test_topk_full_size_plain_workload(sw):
    """The 4,096 best hits of the shortest and a mid-length plain query on the
    full 200,000-sequence database: every score of the row and every hit's
    end compared with the oracle."""
    from conftest import workload, oracle_row
    w = workload("plain")
    with sw.Database(w.residues, w.offsets) as db:
        for qi in (0, 8):
            q = w.queries[qi]
            say("full-size top-k: query %d (m=%d)" % (qi, len(q)))
            hits, scores = db.search_topk(q, w.matrix, 10, 2, k=sw.SW_MAX_TOPK, scores=True)
            want = oracle_row(w, q)
            assert (scores == want).all()
            order = ocpu.top_hits(want, sw.SW_MAX_TOPK)
            assert (hits["seq"] == order).all()
            s, qe, de = ocpu.search_end(q, w.residues, w.offsets, w.matrix, 10, 2, ids=order)
            assert (hits["score"] == s).all()
            assert (hits["query_end"] == qe).all() and (hits["db_end"] == de).all()


@pytest.mark.parametrize("m,go,ge", [(1, 10, 2), (12, 10, 2), (60, 10, 2), (150, 10, 2),
                                     (40, 5, 1), (100, 40, 20), (700, 10, 2), (1500, 10, 2)])
def test_topk_ends_in_column_segments(sw, m, go, ge):
    """Queries against long hit sequences: the end pass runs in column
    segments of 4,096 columns (windows reaching m + ceil(11 m / extend)
    back, more than one segment for the two longest queries, whose early
    windows then start at column 0).  Copies of the query planted to end
    exactly at, just before and just after a segment boundary, and two equal
    copies in different segments of one sequence (the first must be
    reported): every hit's score and end equal the oracle's."""
    rng = np.random.default_rng(80 + m + ge)
    q = swinputs.random_residues(m, rng)
    lengths = np.concatenate([rng.integers(20, 600, 300),
                              [4095, 4096, 4097, 8192, 9000, 20000, 12345]]).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    res = res.copy()
    n = len(lengths)
    big = {int(L): i for i, L in enumerate(lengths) if L >= 4095}
    plants = [(big[8192], 4096 - m), (big[9000], 4096 - m + 1), (big[4097], 4097 - m),
              (big[20000], 5000), (big[20000], 13000), (big[12345], 8191 - m + 1)]
    for sid, at in plants:
        if at >= 0:
            res[offs[sid] + at: offs[sid] + at + m] = q
    say("segmented ends m=%d gaps %d/%d" % (m, go, ge))
    with sw.Database(res, offs) as db:
        hits, scores = db.search_topk(q, B62, go, ge, k=64, scores=True)
    _check_hits(hits, scores, q, res, offs, B62, go, ge, 64)
    if m >= 12:   # the planted copies outscore the rest
        long_hits = [h for h in hits if lengths[h["seq"]] > 4096]
        assert long_hits, "the hits include sequences longer than one segment"
