"""Smith-Waterman protein database search on AMD Instinct MI355X (gfx950).

Python face of libswdb.so (C ABI in include/swdb.h).  `Database` uploads a
protein database once; `search`, `search_batch` and their device-buffer
variants score queries against every database sequence with the library's
HIP kernels.  PyTorch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import _native
from ._native import (SwError, SW_ALPHA, SW_BIN_SEQS, SW_PAD_CODE, SW_MIN_BIN_LEN,
                      SW_DEFAULT_LONG_THRESHOLD, SW_OPT_TIMING, SW_OPT_SAT_LIMIT, SW_OPT_ROWS,
                      SW_OPT_WAVES, SW_OPT_INTRA_ROWS, SW_OPT_INTRA_WAVES, SW_OPT_GRAPHS,
                      SW_OPT_HYBRID_SHARE, SW_OPT_OFFLOAD_BINS,
                      SW_MAX_TOPK, SW_MODE_LOCAL, SW_MODE_GLOBAL, SW_MODE_SEMIGLOBAL)

__all__ = ["Database", "Context", "SwError", "plan", "pack", "host_search", "SW_ALPHA", "SW_BIN_SEQS", "SW_PAD_CODE",
           "SW_MIN_BIN_LEN", "SW_DEFAULT_LONG_THRESHOLD", "SW_OPT_TIMING", "SW_OPT_SAT_LIMIT",
           "SW_OPT_ROWS", "SW_OPT_WAVES", "SW_OPT_INTRA_ROWS", "SW_OPT_INTRA_WAVES", "SW_OPT_GRAPHS",
           "SW_OPT_HYBRID_SHARE", "SW_OPT_OFFLOAD_BINS",
           "SW_MAX_TOPK", "HIT_DTYPE", "ALIGNMENT_DTYPE", "SW_MODE_LOCAL", "SW_MODE_GLOBAL", "SW_MODE_SEMIGLOBAL",
           "MODES"]

# alignment operation names accepted by Database.search_mode
MODES = {"local": SW_MODE_LOCAL, "global": SW_MODE_GLOBAL, "semiglobal": SW_MODE_SEMIGLOBAL}

# one sw_hit: database sequence, score, query end, database end (0-based; -1
# when the score is 0)
HIT_DTYPE = np.dtype([("seq", np.int32), ("score", np.int32), ("query_end", np.int32),
                      ("db_end", np.int32)])
# sw_alignment
ALIGNMENT_DTYPE = np.dtype([("seq", np.int32), ("score", np.int32), ("query_begin", np.int32),
                            ("query_end", np.int32), ("db_begin", np.int32), ("db_end", np.int32),
                            ("ops_offset", np.int64), ("n_ops", np.int32), ("reserved", np.int32)])
_OPS = "MID"


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data if a.size else None
    return a.data_ptr()      # torch tensor


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _matrix(matrix) -> np.ndarray:
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    if m.shape != (SW_ALPHA, SW_ALPHA):
        raise ValueError("matrix must be int8[24, 24]")
    return m


def _check_tensor(t, name: str, dtype_name: str, min_numel: int):
    """Rejects a device buffer the C ABI cannot check itself: not a tensor,
    wrong dtype, non-contiguous or too small (ValueError).  Whether it is in
    GPU memory is checked after every buffer's other properties."""
    import torch
    want = getattr(torch, dtype_name)
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if t.dtype != want:
        raise ValueError("%s must be torch.%s, not %s" % (name, dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < min_numel:
        raise ValueError("%s holds %d elements, needs at least %d" % (name, t.numel(), min_numel))


def _check_on_gpu(**tensors):
    for name, t in tensors.items():
        if not t.is_cuda:
            raise ValueError("%s must be in GPU memory" % name)


def _check_search_args(d_query, d_out, n_seqs: int):
    _check_tensor(d_query, "d_query", "uint8", 0)
    _check_tensor(d_out, "d_out", "int32", n_seqs)
    _check_on_gpu(d_query=d_query, d_out=d_out)


def _check_batch_args(d_queries, qoffs: np.ndarray, d_out, n_seqs: int):
    if qoffs.ndim != 1 or len(qoffs) < 1:
        raise ValueError("query_offsets must be a 1-D array of n_queries + 1 offsets")
    if qoffs[0] != 0 or (np.diff(qoffs) < 0).any():
        raise ValueError("query_offsets must start at 0 and be non-decreasing")
    _check_tensor(d_queries, "d_queries", "uint8", int(qoffs[-1]))
    _check_tensor(d_out, "d_out", "int32", (len(qoffs) - 1) * n_seqs)
    _check_on_gpu(d_queries=d_queries, d_out=d_out)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def plan(offsets, long_threshold: int = 0, residues=None) -> dict:
    """Host-only layout statistics (sw_plan)."""
    offs = _i64(offsets)
    res = _u8(residues) if residues is not None else None
    info = _native.PlanInfo()
    _native.check(_native.lib().sw_plan(_ptr(res), _ptr(offs), len(offs) - 1, long_threshold,
                                        ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in _native.PlanInfo._fields_}


def pack(residues, offsets, long_threshold: int = 0) -> dict:
    """Host-only database layout arrays (sw_pack)."""
    res, offs = _u8(residues), _i64(offsets)
    info = plan(offs, long_threshold, res)
    packed = np.zeros(max(info["packed_dwords"], 1), dtype=np.uint32)
    nb = info["n_bins"] + info["n_long_bins"]
    bins = np.zeros((max(nb, 1), 4), dtype=np.int64)
    slots = np.zeros(max(nb * SW_BIN_SEQS, 1), dtype=np.int32)
    long_ids = np.zeros(max(info["n_long"], 1), dtype=np.int32)
    _native.check(_native.lib().sw_pack(_ptr(res), _ptr(offs), len(offs) - 1, long_threshold,
                                        _ptr(packed), _ptr(bins), _ptr(slots), _ptr(long_ids)))
    return {"info": info, "packed": packed[:info["packed_dwords"]],
            "bins": bins[:nb], "slot_seq": slots[:nb * SW_BIN_SEQS],
            "long_ids": long_ids[:info["n_long"]]}


def host_search(residues, offsets, query, matrix, gap_open: int = 10, gap_extend: int = 2,
                threads: int = 0) -> np.ndarray:
    """Scores with the hybrid search's host scorer alone (sw_host_search):
    host buffers, host threads, no GPU."""
    res, offs, q = _u8(residues), _i64(offsets), _u8(query)
    m = _matrix(matrix)
    out = np.empty(len(offs) - 1, dtype=np.int32)
    _native.check(_native.lib().sw_host_search(_ptr(res), _ptr(offs), len(offs) - 1, _ptr(q),
                                               len(q), _ptr(m), gap_open, gap_extend,
                                               int(threads), _ptr(out)))
    return out


class Database:
    """A protein database resident in device memory (sw_db_load)."""

    def __init__(self, residues, offsets, long_threshold: int = 0):
        L = _native.lib()
        self._res = _u8(residues)
        self._offs = _i64(offsets)
        h = ctypes.c_void_p()
        _native.check(L.sw_db_load_ex(_ptr(self._res), _ptr(self._offs), len(self._offs) - 1,
                                      long_threshold, ctypes.byref(h)))
        self._h = h
        self.n_seqs = len(self._offs) - 1
        self.n_residues = int(self._offs[-1])

    def close(self):
        if getattr(self, "_h", None):
            _native.lib().sw_db_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def info(self) -> dict:
        n, r, ml, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _native.check(_native.lib().sw_db_info(self._h, ctypes.byref(n), ctypes.byref(r),
                                               ctypes.byref(ml), ctypes.byref(nl)))
        return {"n_seqs": n.value, "n_residues": r.value, "max_len": ml.value,
                "n_long": nl.value}

    def set_option(self, key: int, value: int):
        _native.check(_native.lib().sw_set_option(self._h, key, int(value)))

    def stats(self) -> dict:
        st = _native.Stats()
        _native.check(_native.lib().sw_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _native.Stats._fields_}

    def autotune(self, query_lens=None, cache: Optional[str] = None) -> dict:
        """Measures the candidate schedules on this database (sw_autotune_ex)
        for the given query lengths (None: the library's default lengths),
        reading or appending the tuning cache file `cache` if given; returns
        the report.  Later searches use the chosen schedules."""
        rep = _native.TuneReport()
        lens = None if query_lens is None else np.ascontiguousarray(query_lens, dtype=np.int32)
        _native.check(_native.lib().sw_autotune_ex(
            self._h, _ptr(lens), 0 if lens is None else len(lens),
            None if cache is None else str(cache).encode(), ctypes.byref(rep)))
        nb, nc, ni = _native.TUNE_BUCKETS, _native.TUNE_CANDIDATES, _native.TUNE_INTRA_CANDIDATES
        cands = [(rep.cand_rows[c], rep.cand_waves[c]) for c in range(nc)]
        icands = [(rep.intra_cand_rows[c], rep.intra_cand_waves[c]) for c in range(ni)]
        out = []
        for b in range(nb):
            out.append({"query_len": rep.query_len[b],
                        "gcups": {"%dx%d" % cands[c]: rep.gcups[b][c] for c in range(nc)},
                        "batch_gcups": {"%dx%d" % cands[c]: rep.batch_gcups[b][c]
                                        for c in range(nc)},
                        "intra_ms": {"%dx%d" % icands[c]: rep.intra_ms[b][c] for c in range(ni)},
                        "chosen": (rep.rows[b], rep.waves[b]),
                        "batch_chosen": (rep.batch_rows[b], rep.batch_waves[b]),
                        "intra_chosen": (rep.intra_rows[b], rep.intra_waves[b])})
        return {"buckets": out, "from_cache": bool(rep.from_cache)}

    def search(self, query, matrix, gap_open: int = 10, gap_extend: int = 2) -> np.ndarray:
        """Scores of one query against every sequence (host in, host out)."""
        q = _u8(query)
        m = _matrix(matrix)
        out = np.empty(self.n_seqs, dtype=np.int32)
        _native.check(_native.lib().sw_search(self._h, _ptr(q), len(q), _ptr(m), gap_open,
                                              gap_extend, _ptr(out)))
        return out

    def search_async(self, d_query, matrix, gap_open: int, gap_extend: int, d_out,
                     stream=None):
        """Device buffers (torch tensors): d_query uint8[m], d_out int32[n_seqs]."""
        _check_search_args(d_query, d_out, self.n_seqs)
        m = _matrix(matrix)
        _native.check(_native.lib().sw_search_async(
            self._h, _ptr(d_query), int(d_query.numel()), _ptr(m), gap_open, gap_extend,
            _ptr(d_out), _stream_handle(stream)))

    def search_async_noalloc(self, d_query, matrix, gap_open: int, gap_extend: int, d_out,
                             stream=None):
        """As search_async, allocating no device memory (sw_search_async_noalloc):
        its scratch is the library's fixed per-GPU array, so calls on one GPU
        must be ordered (one stream, or events) - overlapping ones race."""
        _check_search_args(d_query, d_out, self.n_seqs)
        m = _matrix(matrix)
        _native.check(_native.lib().sw_search_async_noalloc(
            self._h, _ptr(d_query), int(d_query.numel()), _ptr(m), gap_open, gap_extend,
            _ptr(d_out), _stream_handle(stream)))

    def search_topk(self, query, matrix, gap_open: int = 10, gap_extend: int = 2, k: int = 10,
                    scores: bool = False):
        """The k best hits of one query (sw_search_topk): a structured array
        of HIT_DTYPE, best first, with the end of each hit's best alignment;
        with scores=True also every score (a second return value)."""
        q = _u8(query)
        m = _matrix(matrix)
        kk = max(0, min(int(k), self.n_seqs))
        hits = np.zeros(kk, dtype=HIT_DTYPE)
        out = np.empty(self.n_seqs, dtype=np.int32) if scores else None
        _native.check(_native.lib().sw_search_topk(self._h, _ptr(q), len(q), _ptr(m), gap_open,
                                                   gap_extend, int(k), _ptr(out), _ptr(hits)))
        return (hits, out) if scores else hits

    def traceback(self, query, matrix, gap_open: int = 10, gap_extend: int = 2, seqs=()):
        """Optimal local alignments of the query with the database sequences
        `seqs` (sw_traceback), in that order: a list of dicts with seq,
        score, query_begin/_end, db_begin/_end (0-based inclusive, -1 for a
        score of 0) and ops, the alignment as a string over M (query residue
        against database residue), I (query residue against a gap) and D
        (database residue against a gap)."""
        q = _u8(query)
        m = _matrix(matrix)
        ids = np.ascontiguousarray(seqs, dtype=np.int32)
        out = np.zeros(len(ids), dtype=ALIGNMENT_DTYPE)
        # room for every run (the library checks the indices themselves)
        ok = (ids >= 0) & (ids < self.n_seqs)
        lens = np.where(ok, self._lengths()[np.where(ok, ids, 0)], 0) if len(ids) else \
            np.zeros(0, np.int64)
        cap = int((lens + len(q)).sum())
        ops = np.zeros(max(cap, 1), dtype=np.uint32)
        used = ctypes.c_int64()
        _native.check(_native.lib().sw_traceback(self._h, _ptr(q), len(q), _ptr(m), gap_open,
                                                 gap_extend, _ptr(ids), len(ids), _ptr(out),
                                                 _ptr(ops), cap, ctypes.byref(used)))
        res = []
        for a in out:
            runs = ops[int(a["ops_offset"]):int(a["ops_offset"]) + int(a["n_ops"])]
            res.append({k: int(a[k]) for k in ("seq", "score", "query_begin", "query_end",
                                               "db_begin", "db_end")})
            res[-1]["ops"] = "".join(_OPS[int(r) & 3] * (int(r) >> 2) for r in runs)
        return res

    def _lengths(self):
        if getattr(self, "_lens", None) is None:
            self._lens = np.diff(self._offs)
        return self._lens

    def search_topk_async(self, d_query, matrix, gap_open: int, gap_extend: int, k: int, d_out,
                          d_hits, stream=None):
        """Device buffers (torch tensors): d_query uint8[m], d_out int32[n_seqs],
        d_hits int32[min(k, n_seqs), 4] (rows of seq, score, query end, db end)."""
        _check_search_args(d_query, d_out, self.n_seqs)
        _check_tensor(d_hits, "d_hits", "int32", 4 * max(0, min(int(k), self.n_seqs)))
        _check_on_gpu(d_hits=d_hits)
        m = _matrix(matrix)
        _native.check(_native.lib().sw_search_topk_async(
            self._h, _ptr(d_query), int(d_query.numel()), _ptr(m), gap_open, gap_extend, int(k),
            _ptr(d_out), _ptr(d_hits), _stream_handle(stream)))

    def search_hybrid(self, query, matrix, gap_open: int = 10, gap_extend: int = 2,
                      cpu_threads: int = 0):
        """One query with host cores and the GPU at once (sw_search_hybrid):
        returns (scores, stats)."""
        q = _u8(query)
        m = _matrix(matrix)
        out = np.empty(self.n_seqs, dtype=np.int32)
        st = _native.HybridStats()
        _native.check(_native.lib().sw_search_hybrid(self._h, _ptr(q), len(q), _ptr(m), gap_open,
                                                     gap_extend, int(cpu_threads), _ptr(out),
                                                     ctypes.byref(st)))
        return out, {k: getattr(st, k) for k, _ in _native.HybridStats._fields_}

    def search_mode(self, query, matrix, gap_open: int = 10, gap_extend: int = 2,
                    mode="global") -> np.ndarray:
        """Scores of one query in another alignment mode (sw_search_mode):
        "local", "global" or "semiglobal" (or an SW_MODE_* value)."""
        q = _u8(query)
        m = _matrix(matrix)
        md = MODES[mode] if isinstance(mode, str) else int(mode)
        out = np.empty(self.n_seqs, dtype=np.int32)
        _native.check(_native.lib().sw_search_mode(self._h, _ptr(q), len(q), _ptr(m), gap_open,
                                                   gap_extend, md, _ptr(out)))
        return out

    def search_mode_async(self, d_query, matrix, gap_open: int, gap_extend: int, mode, d_out,
                          stream=None):
        _check_search_args(d_query, d_out, self.n_seqs)
        m = _matrix(matrix)
        md = MODES[mode] if isinstance(mode, str) else int(mode)
        _native.check(_native.lib().sw_search_mode_async(
            self._h, _ptr(d_query), int(d_query.numel()), _ptr(m), gap_open, gap_extend, md,
            _ptr(d_out), _stream_handle(stream)))

    def search_batch(self, queries: Sequence, matrix, gap_open: int = 10,
                     gap_extend: int = 2) -> np.ndarray:
        """Scores of many queries; returns int32[n_queries, n_seqs]."""
        qs = [_u8(q) for q in queries]
        qoffs = np.zeros(len(qs) + 1, dtype=np.int64)
        np.cumsum([len(q) for q in qs], out=qoffs[1:])
        cat = np.concatenate(qs) if qs else np.zeros(0, dtype=np.uint8)
        m = _matrix(matrix)
        out = np.empty((len(qs), self.n_seqs), dtype=np.int32)
        _native.check(_native.lib().sw_search_batch(self._h, _ptr(cat), _ptr(qoffs), len(qs),
                                                    _ptr(m), gap_open, gap_extend, _ptr(out)))
        return out

    def search_batch_async(self, d_queries, query_offsets, matrix, gap_open: int,
                           gap_extend: int, d_out, stream=None):
        qoffs = _i64(query_offsets)
        _check_batch_args(d_queries, qoffs, d_out, self.n_seqs)
        m = _matrix(matrix)
        _native.check(_native.lib().sw_search_batch_async(
            self._h, _ptr(d_queries), _ptr(qoffs), len(qoffs) - 1, _ptr(m), gap_open,
            gap_extend, _ptr(d_out), _stream_handle(stream)))

    def context(self) -> "Context":
        """A new search context: private scratch, so searches on different
        contexts can be in flight at once."""
        return Context(self)

    def context_bytes(self) -> int:
        """Device bytes of fixed scratch one extra context allocates."""
        return int(_native.lib().sw_ctx_bytes(self._h))


class Context:
    """A search context of a Database (sw_ctx_*): device-buffer searches that
    may run concurrently with searches on other contexts."""

    def __init__(self, db: Database):
        h = ctypes.c_void_p()
        _native.check(_native.lib().sw_ctx_create(db._h, ctypes.byref(h)))
        self._h = h
        self.db = db
        self.n_seqs = db.n_seqs

    def close(self):
        if getattr(self, "_h", None):
            _native.lib().sw_ctx_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key: int, value: int):
        _native.check(_native.lib().sw_ctx_set_option(self._h, key, int(value)))

    def stats(self) -> dict:
        st = _native.Stats()
        _native.check(_native.lib().sw_ctx_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _native.Stats._fields_}

    def search_async(self, d_query, matrix, gap_open: int, gap_extend: int, d_out,
                     stream=None):
        _check_search_args(d_query, d_out, self.n_seqs)
        m = _matrix(matrix)
        _native.check(_native.lib().sw_ctx_search_async(
            self._h, _ptr(d_query), int(d_query.numel()), _ptr(m), gap_open, gap_extend,
            _ptr(d_out), _stream_handle(stream)))

    def search_batch_async(self, d_queries, query_offsets, matrix, gap_open: int,
                           gap_extend: int, d_out, stream=None):
        qoffs = _i64(query_offsets)
        _check_batch_args(d_queries, qoffs, d_out, self.n_seqs)
        m = _matrix(matrix)
        _native.check(_native.lib().sw_ctx_search_batch_async(
            self._h, _ptr(d_queries), _ptr(qoffs), len(qoffs) - 1, _ptr(m), gap_open,
            gap_extend, _ptr(d_out), _stream_handle(stream)))
