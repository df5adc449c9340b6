"""GPU parity: library scores vs the CPU oracle, bit-exact.

Every test calls the HIP path through the C ABI (paper_2203_11100_amd ->
libswdb.so) and compares each score with oracle/ (plain scalar Gotoh in C).
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


def _oracle(q, res, offs, S=B62, go=10, ge=2, ids=None):
    return ocpu.search(q, res, offs, S, go, ge, ids=ids)


def _ragged_db(seed=0):
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([
        [0, 0, 1, 2, 3, 4, 5, 7, 8, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257],
        rng.integers(20, 700, 1200),
        [1500, 2100],
    ]).astype(np.int64)
    rng.shuffle(lengths)
    return swinputs.make_database(lengths, rng)


@pytest.mark.parametrize("off", [-1, 0])
def test_plain_small_workload(sw, off):
    w = swinputs.config("plain-small")
    say("plain-small: 2000 seqs, m=144, offload %d" % off)
    with sw.Database(w.residues, w.offsets) as db:
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, off)
        got = db.search(w.queries[0], w.matrix, 10, 2)
    want = _oracle(w.queries[0], w.residues, w.offsets)
    assert (got == want).all(), np.nonzero(got != want)[0][:10]


@pytest.mark.parametrize("off", [0, -1])
@pytest.mark.parametrize("m", [1, 2, 15, 16, 17, 31, 32, 33, 100, 255, 257, 600])
def test_ragged_database_query_lengths(sw, m, off):
    """Every bin in the inter-task kernel (off = 0), or the longest ones
    handed to the long-pair kernel as the search decides (off = -1)."""
    res, offs = _ragged_db()
    q = swinputs.random_residues(m, np.random.default_rng(m))
    say("ragged db, m=%d, offload %d" % (m, off))
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, off)
        got = db.search(q, B62, 10, 2)
    assert (got == _oracle(q, res, offs)).all()


@pytest.mark.parametrize("rows,waves", [(16, 1), (16, 2), (16, 4), (16, 8), (16, 12),
                                        (32, 1), (32, 2), (32, 4), (32, 8),
                                        (12, 12), (14, 12), (18, 12), (20, 12),
                                        (12, 16), (14, 16)])
def test_strip_and_wave_options(sw, rows, waves):
    res, offs = _ragged_db(1)
    q = swinputs.random_residues(333, np.random.default_rng(5))
    say("rows=%d waves=%d" % (rows, waves))
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, 0)     # every bin in the inter-task kernel
        db.set_option(sw.SW_OPT_ROWS, rows)
        db.set_option(sw.SW_OPT_WAVES, waves)
        got = db.search(q, B62, 10, 2)
        st = db.stats()
    assert st["rows"] == rows and st["waves"] == waves
    assert (got == _oracle(q, res, offs)).all()


def test_consecutive_searches_change_schedule(sw):
    """Searches in a row on one database, each with another schedule, query
    length (one strip, several rounds, a single-wave form, an empty query)
    and number of bins handed to the long-pair kernel: the first strip of
    every search reads the boundary rows the previous search left, which
    must be zeros whatever its schedule and whichever bins it skipped."""
    res, offs = _ragged_db(7)
    rng = np.random.default_rng(70)
    plan = [(333, 0, 0, 0), (5, 12, 16, 3), (700, 20, 12, -1), (0, 0, 0, 0), (40, 14, 16, 1),
            (150, 16, 1, 0), (1, 0, 0, 5), (900, 32, 8, 2), (211, 18, 12, 0), (333, 0, 0, -1),
            (333, 0, 0, 0)]
    say("consecutive searches, %d schedules" % len(plan))
    with sw.Database(res, offs) as db:
        for m, rows, waves, off in plan:
            q = swinputs.random_residues(m, rng)
            db.set_option(sw.SW_OPT_ROWS, rows)
            db.set_option(sw.SW_OPT_WAVES, waves)
            db.set_option(sw.SW_OPT_OFFLOAD_BINS, off)
            got = db.search(q, B62, 10, 2)
            want = _oracle(q, res, offs) if m else np.zeros(len(offs) - 1, np.int32)
            assert (got == want).all(), (m, rows, waves, off)


# (rows, waves, efficiency per strip slot) of the library's fitted schedules
_SCHEDS = [(20, 12, 0.835), (18, 12, 0.821), (16, 12, 0.838), (14, 12, 0.810),
           (12, 12, 0.814), (14, 16, 0.868), (12, 16, 0.863)]


def _fit_schedule(m):
    """The schedule the library fits to a query: the fewest
    ceil(strips / W) * W * R / efficiency, first listed on ties."""
    best = None
    for R, W, eff in _SCHEDS:
        strips = -(-m // R)
        cost = -(-strips // W) * W * R / eff
        if best is None or cost < best[0]:
            best = (cost, R, W)
    return best[1], best[2]


@pytest.mark.parametrize("m", [1, 13, 144, 211, 256, 310, 454, 666, 977, 1184, 1736])
def test_fitted_schedule(sw, m):
    """Without options a search takes the fitted (rows, waves) and stays
    exact (ragged last strips, 16-wave bins shorter than 32 chunks)."""
    res, offs = _ragged_db(40)
    q = swinputs.random_residues(m, np.random.default_rng(41))
    say("fitted schedule m=%d" % m)
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, 0)     # every bin in the inter-task kernel
        got = db.search(q, B62, 10, 2)
        st = db.stats()
    assert (st["rows"], st["waves"]) == _fit_schedule(m)
    assert (got == _oracle(q, res, offs)).all()


@pytest.mark.parametrize("intra_rows", [2, 4, 8])
@pytest.mark.parametrize("intra_waves", [1, 2, 4, 8])
@pytest.mark.parametrize("t_long", [1, 100])
def test_intra_task_path(sw, intra_rows, intra_waves, t_long):
    res, offs = _ragged_db(2)
    q = swinputs.random_residues(1700, np.random.default_rng(6))
    say("t_long=%d intra_rows=%d intra_waves=%d" % (t_long, intra_rows, intra_waves))
    with sw.Database(res, offs, long_threshold=t_long) as db:
        assert db.info()["n_long"] > 0
        db.set_option(sw.SW_OPT_INTRA_ROWS, intra_rows)
        db.set_option(sw.SW_OPT_INTRA_WAVES, intra_waves)
        got = db.search(q, B62, 10, 2)
    assert (got == _oracle(q, res, offs)).all()


def _segment_db(seed=12):
    """Long sequences of 500..20,000 residues (lengths at and around
    multiples of 1,000, the segment length for long threshold 500) among
    short ones, one of them an embedded copy target."""
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([rng.integers(20, 499, 300), [500, 999, 1000, 1001, 1999, 2000,
                                                           2001, 3000, 20_000, 12_345],
                              rng.integers(500, 9_000, 40)]).astype(np.int64)
    rng.shuffle(lengths)
    return swinputs.make_database(lengths, rng)


@pytest.mark.parametrize("m,go,ge,segmented", [(1, 10, 2, True), (10, 10, 2, True),
                                                (60, 10, 2, True), (150, 10, 2, True),
                                                (160, 10, 2, False), (83, 10, 1, True),
                                                (84, 12, 1, False), (40, 5, 0, False),
                                                (100, 40, 20, True)])
def test_long_pairs_in_column_segments(sw, m, go, ge, segmented):
    """Short queries score the long pairs in column segments of 1,000
    columns (twice the long threshold) whose windows reach back
    m + ceil(11 m / extend) columns; scores stay exact, including segment
    boundaries, planted copies and every sequence sent to rescoring."""
    res, offs = _segment_db()
    rng = np.random.default_rng(m)
    q = swinputs.random_residues(m, rng)
    # plant the query across a segment boundary of the 20,000-residue sequence
    lens = np.diff(offs)
    big = int(np.nonzero(lens == 20_000)[0][0])
    at = int(offs[big]) + 4_000 - m // 2
    res = res.copy()
    res[at:at + m] = q
    reach = m + (m * 11 + ge - 1) // ge if ge > 0 else None
    say("segments: m=%d gaps %d/%d reach %s" % (m, go, ge, reach))
    want = _oracle(q, res, offs, go=go, ge=ge)
    with sw.Database(res, offs, long_threshold=500) as db:
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, 0)     # the long pairs alone in the pair kernel
        for limit in (32767, 40):
            db.set_option(sw.SW_OPT_SAT_LIMIT, limit)
            got = db.search(q, B62, go, ge)
            st = db.stats()
            assert (got == want).all(), np.nonzero(got != want)[0][:10]
            assert (st["long_overlap"] == reach) if segmented else (st["long_overlap"] == -1)
            n_pairs = (db.info()["n_long"] + 1) // 2
            assert (st["long_items"] > n_pairs) if segmented else (st["long_items"] == n_pairs)
    assert want[big] == sum(int(B62[c, c]) for c in q)


def _bins_db(seed, with_long):
    """Short sequences of every length class (empty ones, a last bin with an
    odd count) and, optionally, a few long ones."""
    rng = np.random.default_rng(seed)
    parts = [[0, 0, 0, 1, 2, 3], rng.integers(1, 60, 200), rng.integers(60, 1200, 500),
             [1999, 2000, 2047]]
    if with_long:
        parts.append([2048, 2600, 4100])
    lengths = np.concatenate(parts).astype(np.int64)
    rng.shuffle(lengths)
    return swinputs.make_database(lengths, rng)


def _bin_pairs(lens, k, t_long):
    """Pairs of neighbouring sequences in the k longest short bins."""
    short = np.sort(lens[lens < t_long])[::-1]
    counts = [min(128, len(short) - 128 * b) for b in range((len(short) + 127) // 128)]
    return sum((c + 1) // 2 for c in counts[:k])


@pytest.mark.parametrize("with_long", [True, False])
@pytest.mark.parametrize("off", [0, 1, 2, 6, 1000, -1])
def test_short_bins_through_the_pair_kernel(sw, with_long, off):
    """The longest short bins handed to the long-pair kernel (two sequences
    per workgroup; an odd bin leaves one alone, two empty sequences score 0
    without reading anything): every score exact, with and without long
    sequences, for a long query (whole pairs) and a short one (the long
    pairs in column segments, each handed-over pair one segment), and with
    the rescoring limit forced low so that the pair kernel's flags reach
    the 32-bit rescoring."""
    res, offs = _bins_db(31, with_long)
    lens = np.diff(offs)
    rng = np.random.default_rng(32)
    t_long = sw.SW_DEFAULT_LONG_THRESHOLD
    # a copy of the long query inside one sequence of the longest bin: a
    # score above the half-precision range
    q = swinputs.random_residues(1300, rng)
    top = int(np.nonzero(lens == 2047)[0][0])
    res = res.copy()
    res[offs[top] + 300:offs[top] + 1600] = q
    for m, qq in ((1300, q), (90, swinputs.random_residues(90, rng))):
        want = _oracle(qq, res, offs)
        with sw.Database(res, offs) as db:
            db.set_option(sw.SW_OPT_OFFLOAD_BINS, off)
            n_long_pairs = (db.info()["n_long"] + 1) // 2
            for limit in (32767, 40):
                say("offload %d, long %s, m=%d, limit %d" % (off, with_long, m, limit))
                db.set_option(sw.SW_OPT_SAT_LIMIT, limit)
                got = db.search(qq, B62, 10, 2)
                st = db.stats()
                assert (got == want).all(), np.nonzero(got != want)[0][:10]
                if limit == 40:
                    assert st["n_rescored"] == int((want >= 40).sum())
                segmented = st["long_items"] > 0 and st["long_overlap"] >= 0
                if off >= 0 and not segmented:
                    assert st["long_items"] == n_long_pairs + _bin_pairs(lens, off, t_long)
                if off == -1 and m == 1300:
                    assert st["long_items"] > n_long_pairs    # the search hands some over


def test_offload_decision_follows_the_database_shape(sw):
    """The automatic choice: a database of many sequences of similar length
    keeps every bin in the inter-task kernel; a long query against a few
    hundred short sequences hands bins over (its longest bin would otherwise
    outlast the rest of the search); both exact on sampled sequences."""
    rng = np.random.default_rng(33)
    res, offs = swinputs.make_database(rng.integers(200, 301, 60_000).astype(np.int64), rng)
    q = swinputs.random_residues(400, rng)
    ids = rng.choice(len(offs) - 1, 200, replace=False)
    with sw.Database(res, offs) as db:
        got = db.search(q, B62, 10, 2)
        st = db.stats()
    assert st["long_items"] == 0
    assert (got[ids] == _oracle(q, res, offs, ids=ids)).all()
    res, offs = swinputs.make_database(
        swinputs.lognormal_lengths(700, 355.0, 0.75, 20, 2000, rng), rng)
    q = swinputs.random_residues(3000, rng)
    with sw.Database(res, offs) as db:
        got = db.search(q, B62, 10, 2)
        st = db.stats()
    assert st["long_items"] > 0
    assert (got == _oracle(q, res, offs)).all()


@pytest.mark.parametrize("limit", [0, 40, 32767])
def test_forced_rescoring(sw, limit):
    res, offs = _ragged_db(3)
    q = swinputs.random_residues(300, np.random.default_rng(7))
    say("sat limit %d" % limit)
    lens = np.diff(offs)
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_SAT_LIMIT, limit)
        got = db.search(q, B62, 10, 2)
        st = db.stats()
        t_long = sw.SW_DEFAULT_LONG_THRESHOLD
    want = _oracle(q, res, offs)
    assert (got == want).all()
    # both packed kernels (bins and the long list) hand scores at or above the
    # limit to the 32-bit rescoring; the exact range of binary16 ends at 2048
    assert (lens >= t_long).any()
    if limit == 0:
        assert st["n_rescored"] == len(lens)
    if limit == 40:
        assert st["n_rescored"] == int((want >= 40).sum())
    if limit == 32767:
        assert st["n_rescored"] == int((want >= 2048).sum())


@pytest.mark.parametrize("off", [0, -1])
def test_scores_around_the_half_precision_limit(sw, off):
    """Planted matches scoring ~1,400..2,500 in the packed kernels' bins:
    every score exact, and exactly those >= 2048 rescored in 32 bits (single
    and batched searches; the single search with every bin in the
    inter-task kernel, or the longest handed to the long-pair kernel)."""
    rng = np.random.default_rng(31)
    W = swinputs.ALPHABET.index("W")
    C = swinputs.ALPHABET.index("C")
    q = np.concatenate([np.full(100, W, np.uint8), np.full(112, C, np.uint8),
                        swinputs.random_residues(40, rng)])
    lengths = rng.integers(50, 600, 400).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    seqs = [res[offs[i]:offs[i + 1]] for i in range(len(lengths))]
    for k, cut in enumerate((0, 3, 6, 9, 14, 20, 30, 45, 60)):
        seqs[7 + 31 * k] = np.concatenate([swinputs.random_residues(12, rng), q[cut:],
                                           swinputs.random_residues(5, rng)])
    lens = np.array([len(x) for x in seqs], dtype=np.int64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    res = np.concatenate(seqs)
    want = _oracle(q, res, offs)
    assert ((want >= 1800) & (want < 2048)).any() and (want > 2048).sum() >= 3
    qs = [q, q[20:].copy(), swinputs.random_residues(90, rng)]
    wants = [_oracle(x, res, offs) for x in qs]
    # all in bins; then the planted ones (>= 257 residues) in the long list,
    # scored by the packed intra-task kernel (batched: long bins)
    for t_long in (10**6, 250):
        say("half-precision limit, long threshold %d, offload %d" % (t_long, off))
        with sw.Database(res, offs, long_threshold=t_long) as db:
            db.set_option(sw.SW_OPT_OFFLOAD_BINS, off)
            if t_long == 250:
                assert db.info()["n_long"] >= 9
            got = db.search(q, B62, 10, 2)
            st = db.stats()
            gotb = db.search_batch(qs, B62, 10, 2)
            stb = db.stats()
        assert (got == want).all()
        assert st["n_rescored"] == int((want >= 2048).sum())
        for row, wq in zip(gotb, wants):
            assert (row == wq).all()
        assert stb["n_rescored"] == sum(int((wq >= 2048).sum()) for wq in wants)


@pytest.mark.parametrize("off", [0, -1])
def test_planted_overflow_in_short_bins(sw, off):
    """Scores above 32767 inside the packed kernels' bins are rescored
    exactly (every bin in the inter-task kernel, or as the search decides)."""
    rng = np.random.default_rng(8)
    W = swinputs.ALPHABET.index("W")
    q = np.concatenate([np.full(2700, W, np.uint8), swinputs.random_residues(1200, rng)])
    lengths = rng.integers(50, 900, 300).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    seqs = [res[offs[i]:offs[i + 1]] for i in range(len(lengths))]
    planted = [5, 77, 200]
    for i in planted:
        seqs[i] = np.concatenate([swinputs.random_residues(30, rng), q, swinputs.random_residues(9, rng)])
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    res = np.concatenate(seqs)
    diag = int(sum(int(B62[c, c]) for c in q))
    assert diag > 32767
    say("planted overflow, offload %d" % off)
    with sw.Database(res, offs, long_threshold=10**6) as db:
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, off)
        got = db.search(q, B62, 10, 2)
        st = db.stats()
    assert st["n_rescored"] >= len(planted)
    for i in planted:
        assert got[i] == diag
    assert (got == _oracle(q, res, offs)).all()


@pytest.mark.parametrize("off", [0, 4])
@pytest.mark.parametrize("gaps", [(0, 0), (5, 5), (11, 1), (40, 1), (1000, 1000), (12, 2),
                                  (3000, 2500), (5000, 1)])
def test_gap_penalties(sw, gaps, off):
    """Gap penalties from none to above the binary16 exact range (passed to
    the packed kernels as 2048), with the four longest bins in either kernel."""
    res, offs = _ragged_db(4)
    q = swinputs.random_residues(180, np.random.default_rng(9))
    say("gaps", gaps, "offload", off)
    with sw.Database(res, offs, long_threshold=1000) as db:
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, off)
        got = db.search(q, B62, *gaps)
    assert (got == _oracle(q, res, offs, B62, *gaps)).all()


def test_random_asymmetric_full_range_matrix(sw):
    rng = np.random.default_rng(10)
    S = rng.integers(-128, 128, size=(24, 24)).astype(np.int8)
    res, offs = _ragged_db(5)
    q = swinputs.random_residues(400, rng)
    say("random matrix")
    with sw.Database(res, offs, long_threshold=1000) as db:
        got = db.search(q, S, 13, 3)
    assert (got == _oracle(q, res, offs, S, 13, 3)).all()


def test_empty_query_and_empty_database(sw):
    res, offs = _ragged_db(6)
    with sw.Database(res, offs) as db:
        got = db.search(np.zeros(0, np.uint8), B62, 10, 2)
    assert (got == 0).all()
    with sw.Database(np.zeros(0, np.uint8), np.zeros(1, np.int64)) as db:
        assert db.search(swinputs.encode("ACDE"), B62, 10, 2).shape == (0,)


def test_very_long_query_and_sequence(sw):
    """A 40,000-residue query (2,858 strips of 14) against bins and a long
    list holding a 60,000-residue sequence, single and batched: exact."""
    rng = np.random.default_rng(50)
    lengths = np.concatenate([rng.integers(1, 3000, 300), [60000, 9000, 2100]]).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    q = swinputs.random_residues(40000, rng)
    q2 = swinputs.random_residues(700, rng)
    say("very long query and sequence")
    want = _oracle(q, res, offs)
    want2 = _oracle(q2, res, offs)
    with sw.Database(res, offs) as db:
        assert db.info()["n_long"] >= 3
        got = db.search(q, B62, 10, 2)
        gotb = db.search_batch([q, q2], B62, 10, 2)
    assert (got == want).all()
    assert (gotb[0] == want).all() and (gotb[1] == want2).all()


def test_batch_and_async_match_single(sw):
    import torch
    res, offs = _ragged_db(7)
    rng = np.random.default_rng(11)
    qs = [swinputs.random_residues(int(m), rng) for m in (0, 50, 144, 700, 31)]
    say("batch/async")
    with sw.Database(res, offs, long_threshold=600) as db:
        single = np.stack([db.search(q, B62, 10, 2) for q in qs])
        batch = db.search_batch(qs, B62, 10, 2)
        assert (single == batch).all()
        cat = torch.from_numpy(np.concatenate(qs)).cuda()
        qoffs = np.zeros(len(qs) + 1, np.int64)
        np.cumsum([len(q) for q in qs], out=qoffs[1:])
        d_out = torch.full((len(qs), db.n_seqs), -1, dtype=torch.int32, device="cuda")
        db.search_batch_async(cat, qoffs, B62, 10, 2, d_out)
        torch.cuda.synchronize()
        assert (d_out.cpu().numpy() == single).all()
        d1 = torch.full((db.n_seqs,), -1, dtype=torch.int32, device="cuda")
        db.search_async(torch.from_numpy(qs[3]).cuda(), B62, 10, 2, d1)
        torch.cuda.synchronize()
        assert (d1.cpu().numpy() == single[3]).all()
    for q, row in zip(qs, single):
        assert (row == _oracle(q, res, offs)).all()


def test_invalid_arguments_write_nothing(sw):
    res, offs = _ragged_db(8)
    L = sw._native.lib()
    with sw.Database(res, offs) as db:
        q = swinputs.encode("ACDEFGHIK")
        out = np.full(db.n_seqs, -7, dtype=np.int32)
        for go, ge in ((2, 3), (-1, 0), ((1 << 30) + 1, 0)):
            rc = L.sw_search(db._h, q.ctypes.data, len(q), B62.ctypes.data, go, ge, out.ctypes.data)
            assert rc in (sw._native.SW_EINVAL, sw._native.SW_ERANGE)
        bad = q.copy(); bad[3] = 24
        rc = L.sw_search(db._h, bad.ctypes.data, len(bad), B62.ctypes.data, 10, 2, out.ctypes.data)
        assert rc == sw._native.SW_EINVAL
        assert (out == -7).all()
        with pytest.raises(sw.SwError):
            db.set_option(sw.SW_OPT_ROWS, 7)


def test_repeatable(sw):
    w = swinputs.config("plain-small")
    with sw.Database(w.residues, w.offsets) as db:
        a = db.search(w.queries[0], w.matrix, 10, 2)
        for _ in range(3):
            assert (db.search(w.queries[0], w.matrix, 10, 2) == a).all()


def test_long_mix_workload_scaled(sw):
    w = swinputs.config("long-mix", scale=0.05)
    qs = [w.queries[0], w.queries[4], w.queries[9]]     # m = 1000, 5000, 10000
    say("long-mix 5%%: %d seqs, %d long" % (w.n_seqs, int((np.diff(w.offsets) >= 10000).sum())))
    with sw.Database(w.residues, w.offsets) as db:
        got = db.search_batch(qs, w.matrix, 10, 2)
    for q, row in zip(qs, got):
        assert (row == _oracle(q, w.residues, w.offsets)).all()
    diag = int(sum(int(B62[c, c]) for c in qs[2]))
    assert diag > 32767
    assert (got[2][w.planted] == diag).all()


def _plain_gpu_rows(sw, w):
    """The 20 plain queries searched as the benchmark does: one asynchronous
    search per query on the current stream, database resident."""
    import torch
    with sw.Database(w.residues, w.offsets) as db:
        outs = []
        for q in w.queries:
            d_out = torch.empty(db.n_seqs, dtype=torch.int32, device="cuda")
            db.search_async(torch.from_numpy(q).cuda(), w.matrix, 10, 2, d_out)
            outs.append(d_out)
        torch.cuda.synchronize()
        return np.stack([o.cpu().numpy() for o in outs])


def _check_bounds(row, q, lens):
    # every score: 0 <= s <= min(m, n) * 11 (the largest BLOSUM62 entry)
    assert (row >= 0).all()
    assert (row <= np.minimum(len(q), lens) * 11).all()


def test_full_size_plain_workload_full_rows(sw):
    """All 20 queries on the full 200,000-sequence database in the launch
    configuration the benchmark times.  Every one of the 200,000 scores of
    the five shortest queries (144..310 residues) is compared with the
    oracle; the other queries are sampled across the length distribution
    (the longest query's full row is the next test)."""
    from conftest import workload, oracle_row
    w = workload("plain")
    lens = np.diff(w.offsets)
    say("full plain workload: %d seqs, %d residues" % (w.n_seqs, w.n_residues))
    got = _plain_gpu_rows(sw, w)
    _PLAIN_GOT["rows"] = got
    for qi in range(5):
        want = oracle_row(w, w.queries[qi])
        bad = np.nonzero(got[qi] != want)[0]
        assert len(bad) == 0, (qi, bad[:5], got[qi][bad[:5]], want[bad[:5]])
        say("query %d (m=%d): all %d scores equal the oracle" % (qi, len(w.queries[qi]), w.n_seqs))
    order = np.argsort(-lens, kind="stable")
    rng = np.random.default_rng(12)
    ids = np.unique(np.concatenate([order[:6], order[-6:], rng.choice(w.n_seqs, 60, replace=False)]))
    import oracle.cpu as ocpu
    for qi, q in enumerate(w.queries):
        _check_bounds(got[qi], q, lens)
        if qi >= 5:
            want = ocpu.search(q, w.residues, w.offsets, w.matrix, 10, 2, ids=ids)
            assert (got[qi][ids] == want).all(), (qi, ids[got[qi][ids] != want][:5])


_PLAIN_GOT = {}


def test_full_size_plain_workload_longest_query_full_row(sw):
    """Every score of the longest plain query (5,478 residues) against the
    full database, compared with the oracle."""
    from conftest import workload, oracle_row
    w = workload("plain")
    got = _PLAIN_GOT.get("rows")
    if got is None:
        got = _plain_gpu_rows(sw, w)
    say("longest plain query: oracle row of %d scores" % w.n_seqs)
    want = oracle_row(w, w.queries[19])
    bad = np.nonzero(got[19] != want)[0]
    assert len(bad) == 0, (bad[:5], got[19][bad[:5]], want[bad[:5]])


# --------------------------------------------------------------- batched form
def _queries(seed, lengths):
    rng = np.random.default_rng(seed)
    return [swinputs.random_residues(int(m), rng) for m in lengths]


@pytest.mark.parametrize("graphs", [0, 1])
def test_batch_matches_oracle(sw, graphs):
    res, offs = _ragged_db(20)
    qs = _queries(21, [0, 1, 17, 144, 145, 600, 33, 1500, 64, 200, 0, 999])   # odd count, empties
    say("batch, graphs=%d" % graphs)
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_GRAPHS, graphs)
        got = db.search_batch(qs, B62, 10, 2)
    for q, row in zip(qs, got):
        assert (row == _oracle(q, res, offs)).all()


@pytest.mark.parametrize("rows,waves", [(16, 4), (16, 8), (16, 12), (32, 4), (32, 8),
                                        (12, 12), (14, 12), (18, 12), (20, 12), (12, 16),
                                        (14, 16)])
def test_batch_strip_options(sw, rows, waves):
    res, offs = _ragged_db(22)
    qs = _queries(23, [300, 280, 90, 31])
    say("batch rows=%d waves=%d" % (rows, waves))
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_ROWS, rows)
        db.set_option(sw.SW_OPT_WAVES, waves)
        got = db.search_batch(qs, B62, 11, 1)
    for q, row in zip(qs, got):
        assert (row == _oracle(q, res, offs, B62, 11, 1)).all()


def test_batch_long_and_rescoring_items(sw):
    """Long list x all queries and the (sequence, query) rescoring list."""
    res, offs = _ragged_db(24)
    qs = _queries(25, [700, 120, 333])
    say("batch long + rescoring")
    for t_long, limit in ((100, 32767), (10**6, 35), (300, 0)):
        with sw.Database(res, offs, long_threshold=t_long) as db:
            db.set_option(sw.SW_OPT_SAT_LIMIT, limit)
            got = db.search_batch(qs, B62, 10, 2)
        for q, row in zip(qs, got):
            assert (row == _oracle(q, res, offs)).all(), (t_long, limit)


def test_batch_all_sequences_very_long(sw):
    """Every sequence in the very-long list (no bins at all): a batch runs
    only the packed long-pair kernel, with each item's own query, and the
    rescoring; an odd count leaves one pair with an empty half; forced
    rescoring (limit 0) and the full exact range."""
    rng = np.random.default_rng(28)
    lengths = rng.integers(100, 1500, 41).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    qs = _queries(29, [60, 700, 1300, 0, 2500])
    info = sw.plan(offs, 1)
    assert info["n_bins"] == 0 and info["n_long_bins"] == 0 and info["n_very_long"] == 41
    say("batch, every sequence very long")
    for limit in (32767, 0):
        with sw.Database(res, offs, long_threshold=1) as db:
            db.set_option(sw.SW_OPT_SAT_LIMIT, limit)
            got = db.search_batch(qs, B62, 10, 2)
        for q, row in zip(qs, got):
            want = _oracle(q, res, offs) if len(q) else np.zeros(len(lengths), np.int32)
            assert (row == want).all(), (limit, len(q))


def test_batch_graph_replays_with_eager_work_between(sw):
    """Replays of the captured batch graph, with single searches and host
    synchronisation between them, each equal to the oracle.  The single
    searches grow the handle's long-sequence scratch (about 100 long pairs
    against the batch's 5 very long items), freeing the block the first
    capture addressed: the graph must be re-captured, not replayed onto the
    freed block (regression test for that use after free)."""
    import torch
    res, offs = _ragged_db(26)
    qs = _queries(27, [150, 400, 90, 260, 51])
    want = np.stack([_oracle(q, res, offs) for q in qs])
    cat = torch.from_numpy(np.concatenate(qs)).cuda()
    qoffs = np.zeros(len(qs) + 1, np.int64)
    np.cumsum([len(q) for q in qs], out=qoffs[1:])
    say("graph replays")
    with sw.Database(res, offs, long_threshold=500) as db:
        db.set_option(sw.SW_OPT_GRAPHS, 0)
        d_eager = torch.full((len(qs), db.n_seqs), -1, dtype=torch.int32, device="cuda")
        db.search_batch_async(cat, qoffs, B62, 10, 2, d_eager)
        torch.cuda.synchronize()
        assert (d_eager.cpu().numpy() == want).all()
        db.set_option(sw.SW_OPT_GRAPHS, 1)
        d_out = torch.full((len(qs), db.n_seqs), -1, dtype=torch.int32, device="cuda")
        for rep in range(4):
            d_out.fill_(-1)
            db.search_batch_async(cat, qoffs, B62, 10, 2, d_out)
            torch.cuda.synchronize()
            assert (d_out.cpu().numpy() == want).all(), rep
            single = db.search(qs[rep], B62, 10, 2)        # eager work between replays
            assert (single == want[rep]).all()


def test_batch_workload_scaled(sw):
    """The batched workload's recipe on a 2% database: 20 + 200 queries."""
    w = swinputs.config("batched", scale=0.02)
    rng = np.random.default_rng(28)
    ids = rng.choice(w.n_seqs, 40, replace=False)
    say("batched 2%%: %d seqs, %d queries" % (w.n_seqs, len(w.queries)))
    with sw.Database(w.residues, w.offsets) as db:
        got = db.search_batch(w.queries, w.matrix, 10, 2)
    for qi in range(0, len(w.queries), 7):
        want = ocpu.search(w.queries[qi], w.residues, w.offsets, w.matrix, 10, 2, ids=ids)
        assert (got[qi][ids] == want).all(), qi


def test_full_size_batched_workload_full_rows(sw):
    """The full batched workload (the 20 plain queries + 200 of 50..5,000
    residues, 220 queries x 200,000 sequences) as the benchmark runs it: one
    batched search planned and captured into a HIP graph, then replayed.
    Every score equals the single-query search of the same query; whole rows
    compared with the oracle: the shortest and the longest query, and both
    halves of the two pairs of shortest queries (queries are paired two per
    lane in length order); every row checked by bounds."""
    import torch
    from conftest import workload, oracle_row
    w = workload("batched")
    lens = np.diff(w.offsets)
    qlens = np.array([len(q) for q in w.queries])
    cat = torch.from_numpy(np.concatenate(w.queries)).cuda()
    qoffs = np.zeros(len(w.queries) + 1, np.int64)
    np.cumsum(qlens, out=qoffs[1:])
    say("full batched workload: %d queries x %d seqs" % (len(w.queries), w.n_seqs))
    with sw.Database(w.residues, w.offsets) as db:
        out = torch.full((len(w.queries), db.n_seqs), -1, dtype=torch.int32, device="cuda")
        db.search_batch_async(cat, qoffs, w.matrix, 10, 2, out)     # plan + capture
        torch.cuda.synchronize()
        out.fill_(-1)
        db.search_batch_async(cat, qoffs, w.matrix, 10, 2, out)     # graph replay
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # every row against the single-query search of the same query (a
        # different kernel, itself compared with the oracle row by row above)
        single = torch.empty(db.n_seqs, dtype=torch.int32, device="cuda")
        for qi, q in enumerate(w.queries):
            db.search_async(cat[qoffs[qi]:qoffs[qi + 1]], w.matrix, 10, 2, single)
            row = single.cpu().numpy()
            bad = np.nonzero(got[qi] != row)[0]
            assert len(bad) == 0, (qi, qlens[qi], bad[:5], got[qi][bad[:5]], row[bad[:5]])
        say("batched: all %d x %d scores equal the single-query searches"
            % (len(w.queries), w.n_seqs))
        del out
    # the library pairs queries in stable length order, longest first
    order = sorted(range(len(qlens)), key=lambda q: -qlens[q])
    pairs = [order[i:i + 2] for i in range(0, len(order), 2)]
    rows = {order[0], order[-1]} | set(pairs[-1]) | set(pairs[-2])
    for qi in sorted(rows, key=lambda q: qlens[q]):
        want = oracle_row(w, w.queries[qi])
        bad = np.nonzero(got[qi] != want)[0]
        assert len(bad) == 0, (qi, qlens[qi], bad[:5], got[qi][bad[:5]], want[bad[:5]])
        say("batched query %d (m=%d): all %d scores equal the oracle" % (qi, qlens[qi], w.n_seqs))
    for qi, q in enumerate(w.queries):
        _check_bounds(got[qi], q, lens)


_TUNE_FORMS = [(0, 0), (20, 12), (18, 12), (16, 12), (14, 12), (12, 12), (14, 16), (12, 16)]
_TUNE_INTRA = [(2, 1), (4, 1), (8, 1), (2, 2), (4, 2), (8, 2), (2, 4), (4, 4), (8, 4), (2, 8),
               (4, 8)]


def test_autotune_then_searches_stay_exact(sw, tmp_path):
    """The autotuner measures every inter-task form and every long-pair
    schedule, for the caller's query lengths; a second handle of the same
    database applies the cached choice without measuring; searches stay exact
    with the tuned schedules (single, batched, and in a context)."""
    res, offs = _ragged_db(30)
    qs = _queries(31, [150, 700, 1300, 2500])
    lens = [len(q) for q in qs]
    cache = str(tmp_path / "tune.txt")
    say("autotune")
    with sw.Database(res, offs) as db:
        rep = db.autotune()
        assert [b["query_len"] for b in rep["buckets"]] == [192, 448, 1280, 4096]
        for b in rep["buckets"]:
            assert b["chosen"] in _TUNE_FORMS and b["batch_chosen"] in _TUNE_FORMS
            assert b["intra_chosen"] in _TUNE_INTRA          # the database has a long sequence
            assert min(b["gcups"].values()) > 0 and min(b["batch_gcups"].values()) > 0
            assert min(b["intra_ms"].values()) > 0
        rep = db.autotune(lens, cache=cache)
        assert not rep["from_cache"]
        assert [b["query_len"] for b in rep["buckets"]] == [150, 700, 1300, 2500]
        chosen = [(b["chosen"], b["batch_chosen"], b["intra_chosen"]) for b in rep["buckets"]]
        single = [db.search(q, B62, 10, 2) for q in qs]
        batch = db.search_batch(qs, B62, 10, 2)
        ctx = db.context()           # contexts inherit the tuned table
        ctx.close()
    assert len(open(cache).read().splitlines()) == 1
    with sw.Database(res, offs) as db:
        rep = db.autotune(lens, cache=cache)
        assert rep["from_cache"]
        assert [(b["chosen"], b["batch_chosen"], b["intra_chosen"])
                for b in rep["buckets"]] == chosen
        again = [db.search(q, B62, 10, 2) for q in qs]
    for q, a, b, c in zip(qs, single, batch, again):
        want = _oracle(q, res, offs)
        assert (a == want).all() and (b == want).all() and (c == want).all()


def test_full_size_long_mix_workload_sampled(sw):
    """The long-sequence mix at full size (50,000 sequences, 2% of 10,000 to
    35,000 residues; 10 queries of 1,000..10,000), single searches and one
    batch: the planted copies of the 10,000-residue query score their closed
    form (> 16 bits), and a sample of short and long sequences is checked by
    the oracle for every query."""
    w = swinputs.config("long-mix")
    lens = np.diff(w.offsets)
    rng = np.random.default_rng(40)
    long_ids = np.nonzero(lens >= 10_000)[0]
    ids = np.unique(np.concatenate([rng.choice(np.nonzero(lens < 10_000)[0], 24, replace=False),
                                    rng.choice(long_ids, 2, replace=False)]))
    diag = int(sum(int(B62[c, c]) for c in w.queries[-1]))
    say("long-mix full: %d seqs, %d residues" % (w.n_seqs, w.n_residues))
    with sw.Database(w.residues, w.offsets) as db:
        single = np.stack([db.search(q, w.matrix, 10, 2) for q in w.queries])
        batch = db.search_batch(w.queries, w.matrix, 10, 2)
    assert (single == batch).all()
    assert diag > 32767 and (single[-1][w.planted] == diag).all()
    from conftest import oracle_row
    for qi, q in enumerate(w.queries):
        if qi < 2:     # m = 1,000 and 2,000: every score
            want = oracle_row(w, q)
            assert (single[qi] == want).all(), (qi, np.nonzero(single[qi] != want)[0][:5])
            say("long mix query %d (m=%d): all %d scores equal the oracle" % (qi, len(q), w.n_seqs))
        else:
            want = ocpu.search(q, w.residues, w.offsets, w.matrix, 10, 2, ids=ids)
            assert (single[qi][ids] == want).all(), qi
