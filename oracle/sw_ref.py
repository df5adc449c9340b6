"""Pure-Python oracle implementations (test infrastructure only).

Both functions follow the Smith-Waterman local alignment score of paper
section 2.2, with the affine gap penalty "10(2)" of section 4.1 read as
w(k) = gap_open + (k - 1) * gap_extend (gap_open is the cost of a one-residue
gap).  Sequences are integer codes indexing the substitution matrix S, with
S[x][y] the score of query residue x against database residue y.
"""
from __future__ import annotations

import itertools
import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np


def gap_cost(k: int, gap_open: int, gap_extend: int) -> int:
    """Cost of a run of k unmatched residues in one sequence; w(0) = 0."""
    if k == 0:
        return 0
    return gap_open + (k - 1) * gap_extend


def _chains(m: int, n: int):
    """Every chain (i_1 < ... < i_r, j_1 < ... < j_r), r >= 1."""
    for r in range(1, min(m, n) + 1):
        for I in itertools.combinations(range(m), r):
            for J in itertools.combinations(range(n), r):
                yield I, J


def sw_bruteforce(a: Sequence[int], b: Sequence[int], S, gap_open: int,
                  gap_extend: int) -> int:
    """Definition of the local alignment score, by enumeration of all chains.

    A local alignment matches residue pairs (i_t, j_t) strictly increasing in
    both sequences; between consecutive matched pairs the skipped residues of
    each sequence form one gap.  Its score is the sum of the matched pairs'
    substitution scores minus the gaps' costs; the empty alignment scores 0.
    Exponential: for tiny inputs only.
    """
    best = 0
    for I, J in _chains(len(a), len(b)):
        s = sum(int(S[a[i]][b[j]]) for i, j in zip(I, J))
        for t in range(len(I) - 1):
            s -= gap_cost(I[t + 1] - I[t] - 1, gap_open, gap_extend)
            s -= gap_cost(J[t + 1] - J[t] - 1, gap_open, gap_extend)
        best = max(best, s)
    return best


def sw_bruteforce_table(a: Sequence[int], b: Sequence[int], S,
                        gaps: Iterable[Tuple[int, int]]) -> List[int]:
    """sw_bruteforce for several (gap_open, gap_extend) pairs at once.

    Each chain is summarised by (substitution sum, number of gaps, residues
    beyond the first in every gap), so that its score under (o, e) is
    sub - n_gaps * o - n_ext * e; the maximum is then taken per (o, e).
    """
    sub, ngap, next_ = [], [], []
    for I, J in _chains(len(a), len(b)):
        sub.append(sum(int(S[a[i]][b[j]]) for i, j in zip(I, J)))
        g = x = 0
        for t in range(len(I) - 1):
            for k in (I[t + 1] - I[t] - 1, J[t + 1] - J[t] - 1):
                if k > 0:
                    g += 1
                    x += k - 1
        ngap.append(g)
        next_.append(x)
    sub = np.array(sub, dtype=np.int64)
    ngap = np.array(ngap, dtype=np.int64)
    next_ = np.array(next_, dtype=np.int64)
    out = []
    for o, e in gaps:
        if len(sub) == 0:
            out.append(0)
        else:
            out.append(int(max(0, (sub - ngap * o - next_ * e).max())))
    return out


def sw_gotoh(a: Sequence[int], b: Sequence[int], S, gap_open: int,
             gap_extend: int) -> int:
    """Gotoh's three-matrix recurrence for the same score, in plain Python.

    With rows i = 1..m over the query and columns j = 1..n over the database
    sequence:
        E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o)      gap along the database
        F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)      gap along the query
        H(i,j) = max(0, H(i-1,j-1) + S(a_i, b_j), E(i,j), F(i,j))
    with H = 0 and E = F = -infinity on the borders; the score is max H.
    """
    m, n = len(a), len(b)
    NEG = -math.inf
    H = [[0] * (n + 1) for _ in range(m + 1)]
    E = [[NEG] * (n + 1) for _ in range(m + 1)]
    F = [[NEG] * (n + 1) for _ in range(m + 1)]
    best = 0
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            E[i][j] = max(E[i][j - 1] - gap_extend, H[i][j - 1] - gap_open)
            F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - gap_open)
            H[i][j] = max(0, H[i - 1][j - 1] + int(S[a[i - 1]][b[j - 1]]),
                          E[i][j], F[i][j])
            best = max(best, H[i][j])
    return int(best)


def sw_bruteforce_end(a: Sequence[int], b: Sequence[int], S, gap_open: int,
                      gap_extend: int) -> Tuple[int, int, int]:
    """Score and end of the best local alignment, by enumeration of all chains.

    The end of a chain is its last matched pair (i_r, j_r).  Several optimal
    chains may end at different pairs; the end reported is the smallest
    (j_r, i_r) in database-then-query order over the optimal chains, as
    0-based residue indices (query, database).  When the score is 0 (no chain
    scores above 0) the end is (-1, -1).  Exponential: tiny inputs only.
    """
    best, end = 0, None
    for I, J in _chains(len(a), len(b)):
        s = sum(int(S[a[i]][b[j]]) for i, j in zip(I, J))
        for t in range(len(I) - 1):
            s -= gap_cost(I[t + 1] - I[t] - 1, gap_open, gap_extend)
            s -= gap_cost(J[t + 1] - J[t] - 1, gap_open, gap_extend)
        if s <= 0:
            continue
        key = (J[-1], I[-1])
        if s > best or (s == best and key < end):
            best, end = s, key
    if best == 0:
        return 0, -1, -1
    return best, end[1], end[0]


def sw_gotoh_end(a: Sequence[int], b: Sequence[int], S, gap_open: int,
                 gap_extend: int) -> Tuple[int, int, int]:
    """Gotoh's recurrence (as in sw_gotoh) with the end of the best alignment.

    The end is the cell (i, j) with H(i, j) equal to the score that comes
    first in database-then-query order (smallest j, then smallest i),
    returned as 0-based residue indices (i - 1, j - 1); (-1, -1) for a
    score of 0.  That cell is the last matched pair of an optimal chain, and
    no optimal chain ends at a smaller (j, i): a cell whose H equals the score
    through E or F has an earlier cell of the same row or column with at
    least that H.
    """
    m, n = len(a), len(b)
    NEG = -math.inf
    H = [[0] * (n + 1) for _ in range(m + 1)]
    E = [[NEG] * (n + 1) for _ in range(m + 1)]
    F = [[NEG] * (n + 1) for _ in range(m + 1)]
    best, end = 0, None
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            E[i][j] = max(E[i][j - 1] - gap_extend, H[i][j - 1] - gap_open)
            F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - gap_open)
            H[i][j] = max(0, H[i - 1][j - 1] + int(S[a[i - 1]][b[j - 1]]),
                          E[i][j], F[i][j])
            if H[i][j] > 0 and (H[i][j] > best or (H[i][j] == best and (j, i) < end)):
                best, end = H[i][j], (j, i)
    if best == 0:
        return 0, -1, -1
    return int(best), end[1] - 1, end[0] - 1


# ------------------------------------------------------- global, semi-global
# Other alignment modes of the same scoring scheme (SW# also offers global
# and semi-global alignment).  Both are maxima over chains of matched pairs
# with the same inner gap costs as the local score; they differ in what the
# residues before the first and after the last matched pair cost:
#   global      : every residue of both sequences is aligned, so the leading
#                 residues of each sequence form one gap each (w(i_1 - 1) and
#                 w(j_1 - 1)), the trailing ones too; the empty chain costs
#                 w(m) + w(n);
#   semi-global : the whole query is aligned within the database sequence:
#                 the query's leading and trailing residues form one gap each,
#                 the database sequence's overhangs are free; the empty chain
#                 costs w(m).
# There is no floor at 0: scores may be negative.
GLOBAL, SEMIGLOBAL = "global", "semiglobal"


def sw_bruteforce_mode(a: Sequence[int], b: Sequence[int], S, gap_open: int, gap_extend: int,
                       mode: str) -> int:
    """Global or semi-global score by enumeration of all chains (tiny inputs)."""
    if mode not in (GLOBAL, SEMIGLOBAL):
        raise ValueError(mode)
    m, n = len(a), len(b)

    def ends(first_i, first_j, last_i, last_j):
        # costs of the unmatched residues before the first and after the
        # last matched pair (0-based indices; -1 / m, n for the empty chain)
        c = gap_cost(first_i, gap_open, gap_extend) + gap_cost(m - 1 - last_i, gap_open, gap_extend)
        if mode == GLOBAL:
            c += gap_cost(first_j, gap_open, gap_extend) + gap_cost(n - 1 - last_j, gap_open,
                                                                     gap_extend)
        return c

    if mode == GLOBAL:
        best = -(gap_cost(m, gap_open, gap_extend) + gap_cost(n, gap_open, gap_extend))
    else:
        best = -gap_cost(m, gap_open, gap_extend)
    for I, J in _chains(m, n):
        s = sum(int(S[a[i]][b[j]]) for i, j in zip(I, J))
        for t in range(len(I) - 1):
            s -= gap_cost(I[t + 1] - I[t] - 1, gap_open, gap_extend)
            s -= gap_cost(J[t + 1] - J[t] - 1, gap_open, gap_extend)
        s -= ends(I[0], J[0], I[-1], J[-1])
        best = max(best, s)
    return best


def sw_gotoh_mode(a: Sequence[int], b: Sequence[int], S, gap_open: int, gap_extend: int,
                  mode: str) -> int:
    """Gotoh's recurrence for the global and semi-global scores.

    As in sw_gotoh but without the 0 in H's maximum, and with borders that
    charge what the mode charges: H(i, 0) = -w(i) (the query's leading
    residues); H(0, j) = -w(j) in global mode, 0 in semi-global mode (free
    leading database residues); E(i, 0) = F(0, j) = -infinity.  The score is
    H(m, n) (global) or max_j H(m, j) (semi-global: free trailing database
    residues); for n = 0 it is H(m, 0).
    """
    if mode not in (GLOBAL, SEMIGLOBAL):
        raise ValueError(mode)
    m, n = len(a), len(b)
    NEG = -math.inf
    w = lambda k: gap_cost(k, gap_open, gap_extend)
    H = [[0] * (n + 1) for _ in range(m + 1)]
    E = [[NEG] * (n + 1) for _ in range(m + 1)]
    F = [[NEG] * (n + 1) for _ in range(m + 1)]
    for i in range(1, m + 1):
        H[i][0] = -w(i)
    for j in range(1, n + 1):
        H[0][j] = -w(j) if mode == GLOBAL else 0
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            E[i][j] = max(E[i][j - 1] - gap_extend, H[i][j - 1] - gap_open)
            F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - gap_open)
            H[i][j] = max(H[i - 1][j - 1] + int(S[a[i - 1]][b[j - 1]]), E[i][j], F[i][j])
    if mode == GLOBAL or n == 0:
        return int(H[m][n])
    return int(max(H[m][j] for j in range(1, n + 1)))


# ---------------------------------------------------------------- traceback
# The alignment behind a local score (SW# computes alignments, section 2.3,
# and a search tool reports them for its best hits).  An alignment is a
# string over M (query residue a_i against database residue b_j), I (a query
# residue against a gap) and D (a database residue against a gap), starting
# at (q_begin, s_begin) and consuming residues left to right; its score is
# the sum of S over the M columns minus w(k) for every maximal run of k I's
# and every maximal run of k D's (a run of I's next to a run of D's is two
# gaps, as between two matched pairs of a chain).


def alignment_score(a: Sequence[int], b: Sequence[int], S, gap_open: int, gap_extend: int,
                    q_begin: int, s_begin: int, ops: str) -> Tuple[int, int, int]:
    """Score of the alignment `ops` placed at (q_begin, s_begin), and the
    0-based indices (q_end, s_end) of the last query and database residues
    it consumes.  Raises ValueError if it runs past either sequence."""
    i, j, score = q_begin, s_begin, 0
    run_op, run_len = "", 0

    def close():
        return -gap_cost(run_len, gap_open, gap_extend) if run_op in ("I", "D") else 0

    for op in ops:
        if op != run_op:
            score += close()
            run_op, run_len = op, 0
        run_len += 1
        if op == "M":
            if i >= len(a) or j >= len(b):
                raise ValueError("alignment runs past a sequence")
            score += int(S[a[i]][b[j]])
            i += 1
            j += 1
        elif op == "I":
            if i >= len(a):
                raise ValueError("alignment runs past the query")
            i += 1
        elif op == "D":
            if j >= len(b):
                raise ValueError("alignment runs past the database sequence")
            j += 1
        else:
            raise ValueError("unknown operation %r" % op)
    score += close()
    return score, i - 1, j - 1


def sw_gotoh_traceback(a: Sequence[int], b: Sequence[int], S, gap_open: int,
                       gap_extend: int) -> Tuple[int, int, int, int, int, str]:
    """An optimal local alignment ending at the end of sw_gotoh_end.

    The recurrence of sw_gotoh over full H, E and F tables, then a walk back
    from the end cell (i, j) (1-based) in three states: in H, stop where
    H(i, j) = 0, else step to (i-1, j-1) emitting M if H came from the
    diagonal, else enter F, else E (the first source in that order that
    equals H); in F emit I and step up, back to H if F came from H(i-1, j) -
    open, else stay in F; in E emit D and step left likewise.  Returns
    (score, q_begin, s_begin, q_end, s_end, ops) with 0-based inclusive
    residue indices; a score of 0 has no alignment: (0, -1, -1, -1, -1, "").
    """
    m, n = len(a), len(b)
    NEG = -math.inf
    H = [[0] * (n + 1) for _ in range(m + 1)]
    E = [[NEG] * (n + 1) for _ in range(m + 1)]
    F = [[NEG] * (n + 1) for _ in range(m + 1)]
    best, end = 0, None
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            E[i][j] = max(E[i][j - 1] - gap_extend, H[i][j - 1] - gap_open)
            F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - gap_open)
            H[i][j] = max(0, H[i - 1][j - 1] + int(S[a[i - 1]][b[j - 1]]),
                          E[i][j], F[i][j])
            if H[i][j] > 0 and (H[i][j] > best or (H[i][j] == best and (j, i) < end)):
                best, end = H[i][j], (j, i)
    if best == 0:
        return 0, -1, -1, -1, -1, ""
    j, i = end
    ops = []
    state = "H"
    while True:
        if state == "H":
            if H[i][j] == 0:
                break
            if H[i][j] == H[i - 1][j - 1] + int(S[a[i - 1]][b[j - 1]]):
                ops.append("M")
                i, j = i - 1, j - 1
            elif H[i][j] == F[i][j]:
                state = "F"
            else:
                state = "E"
        elif state == "F":
            ops.append("I")
            state = "H" if F[i][j] == H[i - 1][j] - gap_open else "F"
            i -= 1
        else:
            ops.append("D")
            state = "H" if E[i][j] == H[i][j - 1] - gap_open else "E"
            j -= 1
    return int(best), i, j, end[1] - 1, end[0] - 1, "".join(reversed(ops))
