"""ctypes wrapper of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.swo_score.restype = I64
        lib.swo_score.argtypes = [P, I64, P, I64, P, ctypes.c_int32, I64, I64]
        lib.swo_search.restype = ctypes.c_int
        lib.swo_search.argtypes = [P, I64, P, P, P, I64, P, ctypes.c_int32, I64, I64, P,
                                   ctypes.c_int32]
        lib.swo_score_mode.restype = I64
        lib.swo_score_mode.argtypes = [P, I64, P, I64, P, ctypes.c_int32, I64, I64, ctypes.c_int32]
        lib.swo_search_mode.restype = ctypes.c_int
        lib.swo_search_mode.argtypes = [P, I64, P, P, P, I64, P, ctypes.c_int32, I64, I64,
                                        ctypes.c_int32, P, ctypes.c_int32]
        lib.swo_score_end.restype = I64
        lib.swo_score_end.argtypes = [P, I64, P, I64, P, ctypes.c_int32, I64, I64, P, P]
        lib.swo_search_end.restype = ctypes.c_int
        lib.swo_search_end.argtypes = [P, I64, P, P, P, I64, P, ctypes.c_int32, I64, I64, P, P,
                                       P, ctypes.c_int32]
        _lib = lib
    return _lib


def default_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    n = os.cpu_count() or 1
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def score(a, b, S, gap_open: int, gap_extend: int) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    S = np.ascontiguousarray(S, dtype=np.int8)
    k = S.shape[0]
    r = _load().swo_score(_ptr(a), len(a), _ptr(b), len(b), _ptr(S), k, gap_open, gap_extend)
    if r < 0:
        raise MemoryError("oracle allocation failed")
    return int(r)


def search(query, residues, offsets, S, gap_open: int, gap_extend: int,
           ids: Optional[np.ndarray] = None, threads: Optional[int] = None) -> np.ndarray:
    """Scores of `query` against every database sequence (or the subset `ids`)."""
    q = np.ascontiguousarray(query, dtype=np.uint8)
    res = np.ascontiguousarray(residues, dtype=np.uint8)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    S = np.ascontiguousarray(S, dtype=np.int8)
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n_items = len(ids)
    else:
        n_items = len(offs) - 1
    out = np.zeros(n_items, dtype=np.int64)
    if n_items == 0:
        return out
    rc = _load().swo_search(_ptr(q), len(q), _ptr(res), _ptr(offs),
                            _ptr(ids) if ids is not None else None, n_items,
                            _ptr(S), S.shape[0], gap_open, gap_extend, _ptr(out),
                            threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle search failed")
    return out


def score_end(a, b, S, gap_open: int, gap_extend: int):
    """(score, query_end, db_end) of the best local alignment: the end is the
    first cell reaching the score in database-then-query order, as 0-based
    residue indices, (-1, -1) for a score of 0."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    S = np.ascontiguousarray(S, dtype=np.int8)
    qe, de = ctypes.c_int64(), ctypes.c_int64()
    r = _load().swo_score_end(_ptr(a), len(a), _ptr(b), len(b), _ptr(S), S.shape[0], gap_open,
                              gap_extend, ctypes.byref(qe), ctypes.byref(de))
    if r < 0:
        raise MemoryError("oracle allocation failed")
    return int(r), int(qe.value), int(de.value)


def search_end(query, residues, offsets, S, gap_open: int, gap_extend: int,
               ids: Optional[np.ndarray] = None, threads: Optional[int] = None):
    """Scores and alignment ends (score_end) of `query` against every
    database sequence or the subset `ids`: three int64 arrays."""
    q = np.ascontiguousarray(query, dtype=np.uint8)
    res = np.ascontiguousarray(residues, dtype=np.uint8)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    S = np.ascontiguousarray(S, dtype=np.int8)
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n_items = len(ids)
    else:
        n_items = len(offs) - 1
    out = np.zeros(n_items, dtype=np.int64)
    qend = np.full(n_items, -1, dtype=np.int64)
    dend = np.full(n_items, -1, dtype=np.int64)
    if n_items == 0:
        return out, qend, dend
    rc = _load().swo_search_end(_ptr(q), len(q), _ptr(res), _ptr(offs),
                                _ptr(ids) if ids is not None else None, n_items,
                                _ptr(S), S.shape[0], gap_open, gap_extend, _ptr(out), _ptr(qend),
                                _ptr(dend), threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle search failed")
    return out, qend, dend


def top_hits(scores, k: int):
    """Indices of the k best scores, best first, ties by smaller index: the
    order of sequences in a top-k result."""
    scores = np.asarray(scores)
    k = min(int(k), len(scores))
    order = np.lexsort((np.arange(len(scores)), -scores.astype(np.int64)))
    return order[:k]


_MODES = {"global": 1, "semiglobal": 2}


def score_mode(a, b, S, gap_open: int, gap_extend: int, mode: str) -> int:
    """Global or semi-global score (see sw_ref.sw_gotoh_mode)."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    S = np.ascontiguousarray(S, dtype=np.int8)
    r = _load().swo_score_mode(_ptr(a), len(a), _ptr(b), len(b), _ptr(S), S.shape[0], gap_open,
                               gap_extend, _MODES[mode])
    if r == np.iinfo(np.int64).min:
        raise MemoryError("oracle allocation failed")
    return int(r)


def search_mode(query, residues, offsets, S, gap_open: int, gap_extend: int, mode: str,
                ids: Optional[np.ndarray] = None, threads: Optional[int] = None) -> np.ndarray:
    """Global or semi-global scores of `query` against every database
    sequence (or the subset `ids`)."""
    q = np.ascontiguousarray(query, dtype=np.uint8)
    res = np.ascontiguousarray(residues, dtype=np.uint8)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    S = np.ascontiguousarray(S, dtype=np.int8)
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n_items = len(ids)
    else:
        n_items = len(offs) - 1
    out = np.zeros(n_items, dtype=np.int64)
    if n_items == 0:
        return out
    rc = _load().swo_search_mode(_ptr(q), len(q), _ptr(res), _ptr(offs),
                                 _ptr(ids) if ids is not None else None, n_items, _ptr(S),
                                 S.shape[0], gap_open, gap_extend, _MODES[mode], _ptr(out),
                                 threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle search failed")
    return out
