"""The half-precision argument behind the packed inter-task kernels, checked
on the CPU.

The kernels evaluate Gotoh's recurrence (E and F kept floored at 0, 3-input
maxima) in IEEE binary16 and rescore in 32-bit integers every sequence whose
half-precision maximum reaches the limit L = min(requested, 2048), with gap
penalties above 2048 passed as 2048.  The claim: a sequence whose true score
is below L comes out exact, and one whose score is L or more comes out >= L.
This model runs the same operations with numpy float16 (whose add, subtract
and maximum of integers of magnitude < 2^24 round once, as the hardware's
do; the single-query kernel forms H_diag + S as a fused multiply-add
(S, 1) * (1, S') + H_diag, whose products by 1 are exact, so it rounds once
exactly as this add does) over a batch of sequences, and compares with the oracle on cases built
to straddle the limit: planted matches scoring 1,900..2,400, a matrix with
entries up to 127, gap penalties above 2048.
"""
import numpy as np
import pytest

import swinputs
from oracle import sw_ref
from oracle import cpu as ocpu

B62 = swinputs.blosum62()
HALF_EXACT = 2048
PAD = -64


def half_scores(q, seqs, matrix, go, ge):
    """binary16 model of the packed kernels' arithmetic: one lane per
    sequence, sequences padded with the pad score."""
    n = max(len(s) for s in seqs)
    b = len(seqs)
    f16 = np.float16
    go_h, ge_h = f16(min(go, HALF_EXACT)), f16(min(ge, HALF_EXACT))
    zero = np.zeros(b, f16)
    # profile values per (row, column, lane)
    cols = np.full((b, n), -1, np.int64)
    for k, s in enumerate(seqs):
        cols[k, :len(s)] = s
    m = len(q)
    H = np.zeros((m, b), f16)     # H of the previous column, per row
    E = np.zeros((m, b), f16)
    best = np.zeros(b, f16)
    for j in range(n):
        c = cols[:, j]
        hd = zero.copy()          # H(i-1, j-1) for row 0
        F = zero.copy()
        for i in range(m):
            p = np.where(c >= 0, matrix[q[i], np.maximum(c, 0)], PAD).astype(f16)
            x = (hd + p).astype(f16)
            h = np.maximum(np.maximum(x, E[i]), F)
            hd = H[i].copy()
            H[i] = h
            best = np.maximum(best, h)
            t = (h - go_h).astype(f16)
            E[i] = np.maximum(np.maximum((E[i] - ge_h).astype(f16), t), zero)
            F = np.maximum(np.maximum((F - ge_h).astype(f16), t), zero)
    return best.astype(np.float64)


def _check(q, seqs, matrix, go, ge, limit=HALF_EXACT):
    res = np.concatenate(seqs)
    offs = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum([len(s) for s in seqs], out=offs[1:])
    exact = ocpu.search(q, res, offs, matrix, go, ge)
    got = half_scores(q, seqs, matrix, go, ge)
    L = min(limit, HALF_EXACT)
    below = exact < L
    assert (got[below] == exact[below]).all(), (got[below], exact[below])
    assert (got[~below] >= L).all(), (got[~below], exact[~below])
    return exact


def _planted(rng, core, n_random, flank=(10, 6)):
    return np.concatenate([swinputs.random_residues(flank[0], rng), core,
                           swinputs.random_residues(flank[1], rng)]).astype(np.uint8)


def test_scores_straddling_2048_blosum62():
    rng = np.random.default_rng(11)
    W = swinputs.ALPHABET.index("W")
    C = swinputs.ALPHABET.index("C")
    # W-W scores 11, C-C 9: cores of 170..220 residues score ~1,900..2,400
    q = np.concatenate([np.full(100, W, np.uint8), np.full(112, C, np.uint8)])
    seqs = []
    for cut in (0, 4, 9, 15, 22, 40, 60):
        seqs.append(_planted(rng, q[cut:], 0))
    seqs += [swinputs.random_residues(int(rng.integers(150, 260)), rng) for _ in range(5)]
    exact = _check(q, seqs, B62, 10, 2)
    assert (exact >= HALF_EXACT).any() and ((exact < HALF_EXACT) & (exact > 1800)).any()
    # above the exact range binary16 does round (2108 comes out as 2104), so
    # those sequences do need the 32-bit rescoring
    got = half_scores(q, seqs, B62, 10, 2)
    assert (got[exact > HALF_EXACT] != exact[exact > HALF_EXACT]).any()


def test_large_matrix_entries_and_lower_limit():
    """Entries up to 127 (the int8 maximum) and a requested limit of 1500:
    exact below the limit, flagged at or above it."""
    rng = np.random.default_rng(12)
    M = B62.astype(np.int16).copy()
    M[17, 17] = 127                  # W-W
    M[4, 4] = 100                    # C-C
    M = M.astype(np.int8)
    W, C = 17, 4
    q = np.concatenate([np.full(14, W, np.uint8), np.full(6, C, np.uint8),
                        swinputs.random_residues(30, rng)])
    seqs = [_planted(rng, q[cut:], 0) for cut in (0, 2, 5, 9, 14, 17)]
    seqs += [swinputs.random_residues(60, rng) for _ in range(3)]
    for limit in (HALF_EXACT, 1500):
        exact = _check(q, seqs, M, 10, 2, limit=limit)
    assert exact.max() > HALF_EXACT


@pytest.mark.parametrize("go,ge", [(3000, 2500), (2048, 2048), (5000, 1), (40, 3)])
def test_gap_penalties_above_the_exact_range(go, ge):
    rng = np.random.default_rng(13)
    q = swinputs.random_residues(60, rng)
    seqs = [swinputs.random_residues(int(rng.integers(20, 90)), rng) for _ in range(8)]
    # gapped near-copies, so gaps matter for small penalties
    for _ in range(3):
        s = q.copy()
        cut = int(rng.integers(5, 50))
        seqs.append(np.concatenate([s[:cut], swinputs.random_residues(4, rng), s[cut:]]))
    _check(q, seqs, B62, go, ge)


def test_model_matches_oracle_on_brute_force_sizes():
    """On tiny inputs the model equals brute force over all alignments."""
    rng = np.random.default_rng(14)
    for _ in range(6):
        q = swinputs.random_residues(int(rng.integers(1, 6)), rng)
        seqs = [swinputs.random_residues(int(rng.integers(1, 6)), rng) for _ in range(4)]
        got = half_scores(q, seqs, B62, 3, 1)
        want = [sw_ref.sw_bruteforce(q, s, B62, 3, 1) for s in seqs]
        assert list(got) == want
