"""Seeded synthetic inputs for protein database search.

This package holds data and random generators only: the residue alphabet,
the BLOSUM62 substitution table, background residue frequencies, the DNA
alphabet with a match/mismatch table, and the workload recipes.  It contains none of the alignment arithmetic, so both the
CPU oracle and the GPU library can draw their inputs from it without sharing
any part of the method.
"""
from .alphabet import ALPHABET, N_CODES, N_STANDARD, encode, decode
from .blosum62 import blosum62
from .background import BACKGROUND_FREQS
from .dna import DNA_ALPHABET, encode_dna, decode_dna, dna_matrix, random_dna
from .workloads import (
    lognormal_lengths,
    random_residues,
    make_database,
    make_query,
    geometric_query_lengths,
    config,
    CONFIG_NAMES,
)

__all__ = [
    "ALPHABET", "N_CODES", "N_STANDARD", "encode", "decode", "blosum62",
    "BACKGROUND_FREQS", "lognormal_lengths", "random_residues", "make_database",
    "make_query", "geometric_query_lengths", "config", "CONFIG_NAMES",
    "DNA_ALPHABET", "encode_dna", "decode_dna", "dna_matrix", "random_dna",
]
