"""Nucleotide alphabet and a match/mismatch scoring table for DNA searches.

SW# aligns DNA as well as protein sequences; the library's arithmetic does
not depend on the alphabet, only on the codes (bytes below 24) and the
caller's substitution table.  DNA uses codes 0..4 for A, C, G, T and N (any
other letter becomes N).  The table scores a match of two bases +match, a
mismatch -mismatch, and anything against N (or a code above 4, which DNA data
never holds) the `n_score`.  The default +5 / -4 is a common nucleotide
scoring; the values are a parameter here, not a published matrix.
"""
import numpy as np

from .alphabet import N_CODES

DNA_ALPHABET = "ACGTN"

_LUT = np.full(256, DNA_ALPHABET.index("N"), dtype=np.uint8)
for _i, _ch in enumerate(DNA_ALPHABET):
    _LUT[ord(_ch)] = _i
    _LUT[ord(_ch.lower())] = _i
_LUT[ord("U")] = _LUT[ord("u")] = DNA_ALPHABET.index("T")   # RNA


def encode_dna(seq: str) -> np.ndarray:
    """Letters -> uint8 codes 0..4 (unknown letters become N)."""
    raw = np.frombuffer(seq.encode("ascii"), dtype=np.uint8)
    return _LUT[raw].copy()


def decode_dna(codes) -> str:
    return "".join(DNA_ALPHABET[int(c)] for c in codes)


def dna_matrix(match: int = 5, mismatch: int = 4, n_score: int = -2) -> np.ndarray:
    """int8[24, 24] table: +match on the diagonal of A, C, G, T, -mismatch
    between two different bases, n_score for N or any higher code."""
    m = np.full((N_CODES, N_CODES), n_score, dtype=np.int8)
    m[:4, :4] = -mismatch
    for i in range(4):
        m[i, i] = match
    return m


def random_dna(n: int, rng: np.random.Generator) -> np.ndarray:
    """n bases drawn uniformly from A, C, G, T (codes 0..3)."""
    return rng.integers(0, 4, size=n, dtype=np.uint8)
