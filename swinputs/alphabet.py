"""Protein residue alphabet in BLOSUM row order.

Codes 0..19 are the 20 standard amino acids (A R N D C Q E G H I L K M F P S T
W Y V), 20..22 are the ambiguity letters B, Z, X and 23 is the stop symbol
'*'.  Every database and query residue crossing the library boundary is one
of these 24 codes, stored as one byte.
"""
import numpy as np

ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"
N_CODES = len(ALPHABET)          # 24
N_STANDARD = 20

_LUT = np.full(256, ALPHABET.index("X"), dtype=np.uint8)
for _i, _ch in enumerate(ALPHABET):
    _LUT[ord(_ch)] = _i
    _LUT[ord(_ch.lower())] = _i
# Rare residues mapped to their closest standard letter.
_LUT[ord("U")] = _LUT[ord("u")] = ALPHABET.index("C")   # selenocysteine
_LUT[ord("O")] = _LUT[ord("o")] = ALPHABET.index("K")   # pyrrolysine
_LUT[ord("J")] = _LUT[ord("j")] = ALPHABET.index("X")


def encode(seq: str) -> np.ndarray:
    """Letters -> uint8 codes (unknown letters become X)."""
    raw = np.frombuffer(seq.encode("ascii"), dtype=np.uint8)
    return _LUT[raw].copy()


def decode(codes) -> str:
    return "".join(ALPHABET[int(c)] for c in codes)
