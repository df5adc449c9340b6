"""Pins of the CPU oracle against what the mathematics fixes.

The paper prints no scores, so the oracle is pinned by: brute-force
enumeration of the definition on tiny inputs (exhaustive over gap penalties,
random non-symmetric matrices), textbook reductions (linear-gap SW, per-diagonal
Kadane, LCS), closed forms under BLOSUM62, hand-derived cases in
tests/golden/hand_cases.txt, and invariants.  Each is chosen so that a dropped
term, a wrong sign or index, a transposed operand or a different gap
convention in the oracle fails at least one test.
"""
import os

import numpy as np
import pytest

import oracle
import oracle.cpu as ocpu
import swinputs

HERE = os.path.dirname(os.path.abspath(__file__))
B62 = swinputs.blosum62()
GAPS_SMALL = [(o, e) for o in range(0, 7) for e in range(0, o + 1)]


# ----------------------------------------------------------------- tiny inputs
def _tiny_cases(seed, count, alpha_max=4, len_max=6):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        k = int(rng.integers(2, alpha_max + 1))
        m = int(rng.integers(0, len_max + 1))
        n = int(rng.integers(0, len_max + 1))
        a = rng.integers(0, k, m).astype(np.uint8)
        b = rng.integers(0, k, n).astype(np.uint8)
        # non-symmetric matrix with mixed signs, sometimes all-negative rows
        S = rng.integers(-6, 7, size=(k, k)).astype(np.int8)
        if rng.random() < 0.2:
            S[int(rng.integers(0, k))] = -rng.integers(1, 5, size=k)
        yield a, b, S


@pytest.mark.parametrize("seed", range(6))
def test_recurrence_equals_definition_bruteforce(seed):
    """Gotoh (Python and C) == chain enumeration, for every 0 <= e <= o <= 6."""
    for a, b, S in _tiny_cases(seed, 25):
        want = oracle.sw_bruteforce_table(a, b, S, GAPS_SMALL)
        for (o, e), w in zip(GAPS_SMALL, want):
            assert oracle.sw_gotoh(a, b, S, o, e) == w, (a, b, S, o, e)
            assert ocpu.score(a, b, S, o, e) == w, (a, b, S, o, e)


def test_bruteforce_table_matches_direct_enumeration():
    for a, b, S in _tiny_cases(99, 20, len_max=5):
        tab = oracle.sw_bruteforce_table(a, b, S, GAPS_SMALL)
        for (o, e), w in zip(GAPS_SMALL, tab):
            assert oracle.sw_bruteforce(a, b, S, o, e) == w


def test_other_gap_convention_by_shifted_open():
    """w(k) = o + k e (open counted on top of every residue) is the oracle with open o + e."""
    rng = np.random.default_rng(7)
    for a, b, S in _tiny_cases(8, 30):
        o = int(rng.integers(0, 6)); e = int(rng.integers(0, 4))
        best = 0
        for I, J in oracle.sw_ref._chains(len(a), len(b)):
            s = sum(int(S[a[i]][b[j]]) for i, j in zip(I, J))
            for t in range(len(I) - 1):
                for k in (I[t + 1] - I[t] - 1, J[t + 1] - J[t] - 1):
                    if k:
                        s -= o + k * e
            best = max(best, s)
        assert ocpu.score(a, b, S, o + e, e) == best


def test_hand_cases():
    n = 0
    with open(os.path.join(HERE, "golden", "hand_cases.txt")) as f:
        for ln in f:
            if not ln.strip() or ln.startswith("#"):
                continue
            q, t, o, e, want = ln.split()
            a, b = swinputs.encode(q), swinputs.encode(t)
            assert oracle.sw_gotoh(a, b, B62, int(o), int(e)) == int(want), ln
            assert ocpu.score(a, b, B62, int(o), int(e)) == int(want), ln
            n += 1
    assert n >= 6


# ------------------------------------------------------- textbook reductions
def _linear_sw(a, b, S, g):
    """Single-matrix Smith-Waterman with linear gap cost g per residue."""
    m, n = len(a), len(b)
    H = np.zeros((m + 1, n + 1), dtype=np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            H[i, j] = max(0, H[i - 1, j - 1] + int(S[a[i - 1]][b[j - 1]]),
                          H[i - 1, j] - g, H[i, j - 1] - g)
    return int(H.max())


def _kadane_diagonals(a, b, S):
    """Best ungapped local alignment: max subarray along every diagonal."""
    best = 0
    m, n = len(a), len(b)
    for d in range(-(m - 1), n):
        run = 0
        for i in range(m):
            j = i + d
            if 0 <= j < n:
                run = max(0, run + int(S[a[i]][b[j]]))
                best = max(best, run)
    return best


def _lcs(a, b):
    m, n = len(a), len(b)
    L = np.zeros((m + 1, n + 1), dtype=np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            L[i, j] = L[i - 1, j - 1] + 1 if a[i - 1] == b[j - 1] else max(L[i - 1, j], L[i, j - 1])
    return int(L[m, n])


def test_equal_open_extend_is_linear_gap_sw():
    rng = np.random.default_rng(11)
    for _ in range(60):
        m, n = rng.integers(0, 40, 2)
        a = rng.integers(0, 20, m).astype(np.uint8)
        b = rng.integers(0, 20, n).astype(np.uint8)
        g = int(rng.integers(0, 9))
        assert ocpu.score(a, b, B62, g, g) == _linear_sw(a, b, B62, g)


def test_prohibitive_gaps_is_per_diagonal_kadane():
    rng = np.random.default_rng(12)
    for _ in range(60):
        m, n = rng.integers(0, 50, 2)
        a = rng.integers(0, 24, m).astype(np.uint8)
        b = rng.integers(0, 24, n).astype(np.uint8)
        big = 11 * 60 + 1
        assert ocpu.score(a, b, B62, big, big) == _kadane_diagonals(a, b, B62)
        assert oracle.sw_gotoh(a, b, B62, big, 0) == _kadane_diagonals(a, b, B62)


def test_free_gaps_unit_match_is_lcs():
    rng = np.random.default_rng(13)
    k = 4
    S = -np.ones((k, k), dtype=np.int8) + 2 * np.eye(k, dtype=np.int8)
    for _ in range(60):
        m, n = rng.integers(0, 40, 2)
        a = rng.integers(0, k, m).astype(np.uint8)
        b = rng.integers(0, k, n).astype(np.uint8)
        assert ocpu.score(a, b, S, 0, 0) == _lcs(a, b)


# ------------------------------------------------ closed forms under BLOSUM62
def test_blosum62_table_shape():
    assert B62.shape == (24, 24) and B62.dtype == np.int8
    assert (B62 == B62.T).all()
    assert B62.min() == -4 and B62.max() == 11
    diag = "A4 R5 N6 D6 C9 Q5 E5 G6 H8 I4 L4 K5 M5 F6 P7 S4 T5 W11 Y7 V4".split()
    for i, d in enumerate(diag):
        assert swinputs.ALPHABET[i] == d[0] and B62[i, i] == int(d[1:])
    s = B62[:20, :20].astype(int)
    # every standard row peaks strictly on the diagonal (needed by the closed forms)
    for x in range(20):
        assert all(s[x, y] < s[x, x] for y in range(20) if y != x)
    assert (B62[23, :23] == -4).all() and B62[23, 23] == 1


def test_self_score_is_diagonal_sum():
    rng = np.random.default_rng(14)
    for m in (1, 2, 5, 50, 300):
        q = swinputs.random_residues(m, rng)
        want = int(sum(int(B62[c, c]) for c in q))
        assert ocpu.score(q, q, B62, 10, 2) == want
        if m <= 50:
            assert oracle.sw_gotoh(q, q, B62, 10, 2) == want


def test_embedded_copy_is_diagonal_sum():
    rng = np.random.default_rng(15)
    for m in (3, 40, 400):
        q = swinputs.random_residues(m, rng)
        x = swinputs.random_residues(int(rng.integers(0, 300)), rng)
        y = swinputs.random_residues(int(rng.integers(0, 300)), rng)
        t = np.concatenate([x, q, y])
        want = int(sum(int(B62[c, c]) for c in q))
        assert ocpu.score(q, t, B62, 10, 2) == want
        assert ocpu.score(t, q, B62, 10, 2) == want


def test_score_beyond_16_bits():
    """A 3,000-residue W run against itself scores 33,000 > 32,767."""
    q = np.full(3000, swinputs.ALPHABET.index("W"), dtype=np.uint8)
    assert ocpu.score(q, q, B62, 10, 2) == 33000


# ----------------------------------------------------------------- invariants
def test_invariants():
    rng = np.random.default_rng(16)
    for _ in range(80):
        m, n = rng.integers(0, 60, 2)
        a = rng.integers(0, 24, m).astype(np.uint8)
        b = rng.integers(0, 24, n).astype(np.uint8)
        o = int(rng.integers(0, 15)); e = int(rng.integers(0, o + 1))
        s = ocpu.score(a, b, B62, o, e)
        assert s >= 0
        assert s == ocpu.score(b, a, B62, o, e)                    # swap (symmetric S)
        assert s == ocpu.score(a[::-1].copy(), b[::-1].copy(), B62, o, e)   # reversal
        lo = max([0] + [int(B62[x, y]) for x in set(a.tolist()) for y in set(b.tolist())])
        assert lo <= s <= min(m, n) * 11
        if n > 2:   # substring monotonicity
            assert ocpu.score(a, b[1:-1], B62, o, e) <= s


def test_empty_inputs_score_zero():
    a = np.zeros(0, dtype=np.uint8)
    b = swinputs.encode("ACDEFG")
    assert ocpu.score(a, b, B62, 10, 2) == 0
    assert ocpu.score(b, a, B62, 10, 2) == 0
    assert oracle.sw_gotoh(a, b, B62, 10, 2) == 0


def test_c_recurrence_matches_python_recurrence_midsize():
    rng = np.random.default_rng(17)
    for _ in range(40):
        m, n = rng.integers(0, 70, 2)
        a = swinputs.random_residues(m, rng)
        b = swinputs.random_residues(n, rng)
        o = int(rng.integers(0, 15)); e = int(rng.integers(0, o + 1))
        assert ocpu.score(a, b, B62, o, e) == oracle.sw_gotoh(a, b, B62, o, e)


def test_threaded_search_matches_single_scores():
    w = swinputs.config("plain-small")
    q = w.queries[0][:60]
    ids = np.arange(0, w.n_seqs, 37)
    got = ocpu.search(q, w.residues, w.offsets, w.matrix, 10, 2, ids=ids, threads=4)
    for t, sid in enumerate(ids[:20]):
        assert got[t] == ocpu.score(q, w.seq(int(sid)), w.matrix, 10, 2)
    full = ocpu.search(q, w.residues, w.offsets, w.matrix, 10, 2, threads=3)
    assert (full[ids] == got).all()


# ------------------------------------------------------------ alignment ends
def _tie_heavy_cases(seed, count):
    """Tiny inputs over 2-3 letters with scores in {-1, 0, 1, 2}: many
    optimal alignments, so the tie-break decides the end."""
    rng = np.random.default_rng(seed)
    for _ in range(count):
        k = int(rng.integers(2, 4))
        a = rng.integers(0, k, int(rng.integers(0, 7))).astype(np.uint8)
        b = rng.integers(0, k, int(rng.integers(0, 7))).astype(np.uint8)
        S = rng.integers(-1, 3, size=(k, k)).astype(np.int8)
        yield a, b, S


@pytest.mark.parametrize("seed", range(4))
def test_end_recurrence_equals_definition_bruteforce(seed):
    """(score, query end, db end): brute force over chains == Gotoh in Python
    == the C oracle, on tie-heavy and general tiny inputs."""
    rng = np.random.default_rng(100 + seed)
    cases = list(_tie_heavy_cases(seed, 30)) + list(_tiny_cases(50 + seed, 15))
    for a, b, S in cases:
        for idx in rng.choice(len(GAPS_SMALL), 5, replace=False):
            o, e = GAPS_SMALL[idx]
            want = oracle.sw_bruteforce_end(a, b, S, o, e)
            assert oracle.sw_gotoh_end(a, b, S, o, e) == want, (a, b, S, o, e)
            assert ocpu.score_end(a, b, S, o, e) == want, (a, b, S, o, e)
            assert want[0] == oracle.sw_bruteforce(a, b, S, o, e)


def test_end_hand_cases():
    n = 0
    with open(os.path.join(HERE, "golden", "hand_ends.txt")) as f:
        for ln in f:
            if not ln.strip() or ln.startswith("#"):
                continue
            q, t, o, e, sc, qe, de = ln.split()
            a, b = swinputs.encode(q), swinputs.encode(t)
            want = (int(sc), int(qe), int(de))
            assert oracle.sw_gotoh_end(a, b, B62, int(o), int(e)) == want, ln
            assert ocpu.score_end(a, b, B62, int(o), int(e)) == want, ln
            n += 1
    assert n >= 5


def test_end_embedded_copy_closed_form():
    """A query copied into a random sequence x q y scores sum S(q_i, q_i)
    (BLOSUM62's rows peak strictly on the diagonal, so only an exact,
    ungapped copy reaches it) and ends at the copy's last residue; with two
    copies the first one's end is reported."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        m = int(rng.integers(20, 60))
        q = swinputs.random_residues(m, rng)
        x = swinputs.random_residues(int(rng.integers(0, 80)), rng)
        y = swinputs.random_residues(int(rng.integers(0, 80)), rng)
        z = swinputs.random_residues(int(rng.integers(0, 30)), rng)
        diag = int(sum(int(B62[c, c]) for c in q))
        t1 = np.concatenate([x, q, y])
        assert ocpu.score_end(q, t1, B62, 10, 2) == (diag, m - 1, len(x) + m - 1)
        t2 = np.concatenate([x, q, z, q, y])
        assert ocpu.score_end(q, t2, B62, 10, 2) == (diag, m - 1, len(x) + m - 1)
        qs = q[:25]
        assert oracle.sw_gotoh_end(qs, np.concatenate([x[:10], qs, y[:5]]), B62, 10, 2) == \
            (int(sum(int(B62[c, c]) for c in qs)), len(qs) - 1, min(len(x), 10) + len(qs) - 1)


# ------------------------------------------------------------------ traceback
def test_alignment_score_hand_cases():
    """The score of an M/I/D string by hand: BLOSUM62 W/W = 11, G/W = -2,
    A/A = 4; gaps 10(2): w(1) = 10, w(3) = 14."""
    e = swinputs.encode
    # WWGWW vs WWWW: MMIMM = 4 x 11 - w(1) = 34, ending at (4, 3)
    assert oracle.alignment_score(e("WWGWW"), e("WWWW"), B62, 10, 2, 0, 0, "MMIMM") == (34, 4, 3)
    # the same residues all matched: MMMM over WWGW/WWWW = 33 - 2 = 31
    assert oracle.alignment_score(e("WWGWW"), e("WWWW"), B62, 10, 2, 0, 0, "MMMM") == (31, 3, 3)
    # a run of three D's is one gap of 3 (14), not three of 1 (30)
    assert oracle.alignment_score(e("AA"), e("AGGGA"), B62, 10, 2, 0, 0, "MDDDM") == (8 - 14, 1, 4)
    # I next to D: two gaps of 1
    assert oracle.alignment_score(e("AGA"), e("AGA"), B62, 10, 2, 0, 0, "MIDM") == (8 - 20, 2, 2)
    # placed after leading residues
    assert oracle.alignment_score(e("KAA"), e("GGAA"), B62, 10, 2, 1, 2, "MM") == (8, 2, 3)
    with pytest.raises(ValueError):
        oracle.alignment_score(e("AA"), e("A"), B62, 10, 2, 0, 0, "MM")
    with pytest.raises(ValueError):
        oracle.alignment_score(e("AA"), e("AA"), B62, 10, 2, 0, 0, "MMX")


@pytest.mark.parametrize("seed", range(4))
def test_traceback_is_an_optimal_alignment_bruteforce(seed):
    """The traceback's alignment, scored from its definition, reaches the
    brute-force optimum, ends at the brute-force end (smallest (j, i) among
    optimal chains) and starts and ends with a matched pair; a score of 0
    has no alignment."""
    rng = np.random.default_rng(300 + seed)
    cases = list(_tie_heavy_cases(200 + seed, 30)) + list(_tiny_cases(250 + seed, 20))
    for a, b, S in cases:
        for idx in rng.choice(len(GAPS_SMALL), 5, replace=False):
            o, e = GAPS_SMALL[idx]
            best, qe, de = oracle.sw_bruteforce_end(a, b, S, o, e)
            score, qb, sb, qe2, de2, ops = oracle.sw_gotoh_traceback(a, b, S, o, e)
            assert (score, qe2, de2) == (best, qe, de), (a, b, S, o, e)
            if best == 0:
                assert (qb, sb, ops) == (-1, -1, "")
                continue
            assert ops[0] == "M" and ops[-1] == "M"
            assert oracle.alignment_score(a, b, S, o, e, qb, sb, ops) == (best, qe, de)


def test_traceback_hand_and_closed_forms():
    """WWGWW / WWWW: the G is skipped (34, MMIMM); an embedded copy of the
    query aligns ungapped from the copy's first residue; a copy with one
    residue deleted from the database side aligns with a single I."""
    e = swinputs.encode
    assert oracle.sw_gotoh_traceback(e("WWGWW"), e("WWWW"), B62, 10, 2) == \
        (34, 0, 0, 4, 3, "MMIMM")
    rng = np.random.default_rng(12)
    for _ in range(10):
        m = int(rng.integers(20, 50))
        q = swinputs.random_residues(m, rng)
        x = swinputs.random_residues(int(rng.integers(0, 40)), rng)
        y = swinputs.random_residues(int(rng.integers(0, 40)), rng)
        diag = int(sum(int(B62[c, c]) for c in q))
        assert oracle.sw_gotoh_traceback(q, np.concatenate([x, q, y]), B62, 10, 2) == \
            (diag, 0, len(x), m - 1, len(x) + m - 1, "M" * m)
    # W-runs around a deleted residue: WWWWWWKWWWWWW against WWWWWWWWWWWW
    # loses the K (w(1) = 10) and keeps 12 W/W pairs (132): 122 with one I
    q = e("WWWWWWKWWWWWW")
    t = e("WWWWWWWWWWWW")
    score, qb, sb, qe, de, ops = oracle.sw_gotoh_traceback(q, t, B62, 10, 2)
    assert score == 122 and ops.count("I") == 1 and ops.count("D") == 0 and ops.count("M") == 12
    assert oracle.alignment_score(q, t, B62, 10, 2, qb, sb, ops) == (122, qe, de)


def test_search_end_matches_per_sequence():
    rng = np.random.default_rng(12)
    lengths = rng.integers(0, 300, 400)
    res, offs = swinputs.make_database(lengths, rng)
    q = swinputs.random_residues(120, rng)
    sc, qe, de = ocpu.search_end(q, res, offs, B62, 10, 2, threads=4)
    assert (sc == ocpu.search(q, res, offs, B62, 10, 2)).all()
    for i in range(0, 400, 13):
        assert (sc[i], qe[i], de[i]) == ocpu.score_end(q, res[offs[i]:offs[i + 1]], B62, 10, 2)
    assert ((qe == -1) == (sc == 0)).all() and ((de == -1) == (sc == 0)).all()
    ids = np.array([5, 3, 399, 0])
    sub = ocpu.search_end(q, res, offs, B62, 10, 2, ids=ids)
    for t in range(3):
        assert (sub[t] == (sc, qe, de)[t][ids]).all()


def test_top_hits_order():
    s = np.array([5, 9, 0, 9, 5, 7, 9, 0])
    assert ocpu.top_hits(s, 5).tolist() == [1, 3, 6, 5, 0]
    assert ocpu.top_hits(s, 100).tolist() == [1, 3, 6, 5, 0, 4, 2, 7]
    assert ocpu.top_hits(s, 0).tolist() == []


# ------------------------------------------------- global and semi-global modes
MODES = (oracle.GLOBAL, oracle.SEMIGLOBAL)


@pytest.mark.parametrize("seed", range(3))
def test_modes_recurrence_equals_definition_bruteforce(seed):
    """Global and semi-global: chain enumeration == Gotoh in Python == C."""
    rng = np.random.default_rng(200 + seed)
    for a, b, S in list(_tiny_cases(300 + seed, 25)) + list(_tie_heavy_cases(400 + seed, 10)):
        for idx in rng.choice(len(GAPS_SMALL), 5, replace=False):
            o, e = GAPS_SMALL[idx]
            for mode in MODES:
                want = oracle.sw_bruteforce_mode(a, b, S, o, e, mode)
                assert oracle.sw_gotoh_mode(a, b, S, o, e, mode) == want, (a, b, S, o, e, mode)
                assert ocpu.score_mode(a, b, S, o, e, mode) == want, (a, b, S, o, e, mode)


def _nw_linear(a, b, S, g):
    """Needleman-Wunsch with linear gap cost g per residue (one matrix)."""
    m, n = len(a), len(b)
    H = np.zeros((m + 1, n + 1), dtype=np.int64)
    H[:, 0] = -g * np.arange(m + 1)
    H[0, :] = -g * np.arange(n + 1)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            H[i, j] = max(H[i - 1, j - 1] + int(S[a[i - 1]][b[j - 1]]), H[i - 1, j] - g,
                          H[i, j - 1] - g)
    return int(H[m, n])


def test_global_linear_gaps_is_needleman_wunsch():
    rng = np.random.default_rng(21)
    for _ in range(40):
        a = swinputs.random_residues(int(rng.integers(0, 30)), rng)
        b = swinputs.random_residues(int(rng.integers(0, 30)), rng)
        g = int(rng.integers(0, 12))
        assert ocpu.score_mode(a, b, B62, g, g, "global") == _nw_linear(a, b, B62, g)


def test_modes_closed_forms():
    """BLOSUM62 rows peak strictly on the diagonal, so: a sequence against
    itself scores sum S(q_i, q_i) globally; against a prefix of itself
    missing k residues, that prefix's sum minus one gap w(k) (global and
    semi-global); a query copied into flanks scores its diagonal sum
    semi-globally; an empty database sequence costs w(m)."""
    rng = np.random.default_rng(22)
    w = lambda k: 0 if k == 0 else 10 + 2 * (k - 1)
    for _ in range(25):
        m = int(rng.integers(1, 80))
        q = swinputs.random_residues(m, rng)
        diag = lambda s: int(sum(int(B62[c, c]) for c in s))
        assert ocpu.score_mode(q, q, B62, 10, 2, "global") == diag(q)
        k = int(rng.integers(0, m))
        for mode in MODES:
            assert ocpu.score_mode(q, q[:m - k], B62, 10, 2, mode) == diag(q[:m - k]) - w(k)
            assert ocpu.score_mode(q, np.zeros(0, np.uint8), B62, 10, 2, mode) == -w(m)
        x = swinputs.random_residues(int(rng.integers(0, 50)), rng)
        y = swinputs.random_residues(int(rng.integers(0, 50)), rng)
        assert ocpu.score_mode(q, np.concatenate([x, q, y]), B62, 10, 2, "semiglobal") == diag(q)
    assert ocpu.score_mode(np.zeros(0, np.uint8), q, B62, 10, 2, "semiglobal") == 0
    assert ocpu.score_mode(np.zeros(0, np.uint8), q, B62, 10, 2, "global") == -w(len(q))


def test_modes_invariants():
    """Swap symmetry (global, symmetric matrix), reversal invariance (both),
    and local >= semi-global >= global for the same inputs."""
    rng = np.random.default_rng(23)
    for _ in range(40):
        a = swinputs.random_residues(int(rng.integers(0, 60)), rng)
        b = swinputs.random_residues(int(rng.integers(0, 60)), rng)
        o = int(rng.integers(0, 14)); e = int(rng.integers(0, o + 1))
        g = ocpu.score_mode(a, b, B62, o, e, "global")
        s = ocpu.score_mode(a, b, B62, o, e, "semiglobal")
        assert g == ocpu.score_mode(b, a, B62, o, e, "global")
        assert g == ocpu.score_mode(a[::-1], b[::-1], B62, o, e, "global")
        assert s == ocpu.score_mode(a[::-1], b[::-1], B62, o, e, "semiglobal")
        assert ocpu.score(a, b, B62, o, e) >= s >= g


def test_search_mode_matches_per_sequence():
    rng = np.random.default_rng(24)
    res, offs = swinputs.make_database(rng.integers(0, 200, 300), rng)
    q = swinputs.random_residues(90, rng)
    for mode in MODES:
        got = ocpu.search_mode(q, res, offs, B62, 10, 2, mode, threads=4)
        for i in range(0, 300, 11):
            assert got[i] == ocpu.score_mode(q, res[offs[i]:offs[i + 1]], B62, 10, 2, mode)


# ------------------------------------------------------------------------ DNA
# DNA searches use codes 0..4 (A C G T N) and a match/mismatch table; the
# oracle's arithmetic is the same, so these pin the table and the closed
# forms that hold for nucleotide scoring.
def test_dna_table_and_encoding():
    D = swinputs.dna_matrix(5, 4, -2)
    assert D.shape == (24, 24) and (D == D.T).all()
    assert all(D[i, i] == 5 for i in range(4))
    assert all(D[i, j] == -4 for i in range(4) for j in range(4) if i != j)
    assert (D[4, :] == -2).all() and (D[:, 4] == -2).all()
    assert list(swinputs.encode_dna("ACGTNacgtuX")) == [0, 1, 2, 3, 4, 0, 1, 2, 3, 3, 4]
    assert swinputs.decode_dna(swinputs.encode_dna("GATTACA")) == "GATTACA"


def test_dna_self_and_embedded_copy_closed_form():
    """Match +5 beats every mismatch and gap, so a base sequence against
    itself, or against any sequence that contains it, scores 5 per base."""
    rng = np.random.default_rng(21)
    D = swinputs.dna_matrix(5, 4, -2)
    for m in (1, 7, 60, 333):
        q = swinputs.random_dna(m, rng)
        assert ocpu.score(q, q, D, 10, 2) == 5 * m
        t = np.concatenate([swinputs.random_dna(int(rng.integers(0, 90)), rng), q,
                            swinputs.random_dna(int(rng.integers(0, 90)), rng)])
        assert ocpu.score(q, t, D, 16, 4) == 5 * m
        assert oracle.sw_gotoh(q[:40], t, D, 16, 4) == 5 * min(m, 40)


def test_dna_unit_match_prohibitive_rest_is_longest_common_substring():
    """Match 1, mismatch and N -100, gaps beyond any gain: the score is the
    length of the longest common substring (checked by direct search)."""
    rng = np.random.default_rng(22)
    D = swinputs.dna_matrix(1, 100, -100)
    for _ in range(40):
        a = swinputs.random_dna(int(rng.integers(0, 25)), rng)
        b = swinputs.random_dna(int(rng.integers(0, 25)), rng)
        best = 0
        for i in range(len(a)):
            for j in range(len(b)):
                k = 0
                while i + k < len(a) and j + k < len(b) and a[i + k] == b[j + k]:
                    k += 1
                best = max(best, k)
        assert ocpu.score(a, b, D, 100, 100) == best
        assert oracle.sw_bruteforce(a[:6], b[:6], D, 100, 100) == ocpu.score(a[:6], b[:6], D, 100, 100)
