"""ctypes binding of libswdb.so (argument marshalling only).

Every step of a search runs in the library's HIP kernels; this module only
converts Python/NumPy/torch arguments to the C ABI declared in
include/swdb.h and turns status codes into exceptions.  It raises if the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswdb.so")

SW_OK, SW_EINVAL, SW_ERANGE, SW_ENOMEM, SW_EDEVICE, SW_EBUSY = range(6)
SW_ALPHA = 24
SW_BIN_SEQS = 128
SW_PAD_CODE = 24
SW_MIN_BIN_LEN = 96
SW_DEFAULT_LONG_THRESHOLD = 2048
SW_OPT_TIMING, SW_OPT_SAT_LIMIT, SW_OPT_ROWS, SW_OPT_WAVES, SW_OPT_INTRA_ROWS = 1, 2, 3, 4, 5
SW_OPT_INTRA_WAVES = 6
SW_OPT_GRAPHS = 7
SW_OPT_HYBRID_SHARE = 8
SW_OPT_OFFLOAD_BINS = 9
SW_MAX_TOPK = 4096
SW_NOALLOC_SCRATCH_BYTES = 128 << 20
SW_MODE_LOCAL, SW_MODE_GLOBAL, SW_MODE_SEMIGLOBAL = 0, 1, 2

_STATUS_NAMES = {1: "SW_EINVAL", 2: "SW_ERANGE", 3: "SW_ENOMEM", 4: "SW_EDEVICE", 5: "SW_EBUSY"}


class SwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int64), ("n_long_bins", ctypes.c_int64),
                ("n_long", ctypes.c_int64), ("n_very_long", ctypes.c_int64),
                ("packed_dwords", ctypes.c_int64), ("boundary_bytes", ctypes.c_int64),
                ("max_len", ctypes.c_int32), ("max_bin_len", ctypes.c_int32),
                ("max_long_len", ctypes.c_int32), ("long_threshold", ctypes.c_int32),
                ("very_long_threshold", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_float), ("ms_inter", ctypes.c_float),
                ("ms_intra", ctypes.c_float), ("ms_rescore", ctypes.c_float),
                ("n_inter_launches", ctypes.c_int32), ("n_rescored", ctypes.c_int32),
                ("inter_cells", ctypes.c_int64), ("intra_cells", ctypes.c_int64),
                ("rows", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("long_items", ctypes.c_int32), ("long_overlap", ctypes.c_int32)]


class HybridStats(ctypes.Structure):
    _fields_ = [("gpu_bins", ctypes.c_int64), ("cpu_seqs", ctypes.c_int64),
                ("gpu_cells", ctypes.c_int64), ("cpu_cells", ctypes.c_int64),
                ("cpu_threads", ctypes.c_int32), ("ms", ctypes.c_float)]


TUNE_BUCKETS, TUNE_CANDIDATES, TUNE_INTRA_CANDIDATES = 4, 8, 11


class TuneReport(ctypes.Structure):
    _fields_ = [("query_len", ctypes.c_int32 * TUNE_BUCKETS),
                ("cand_rows", ctypes.c_int32 * TUNE_CANDIDATES),
                ("cand_waves", ctypes.c_int32 * TUNE_CANDIDATES),
                ("gcups", (ctypes.c_float * TUNE_CANDIDATES) * TUNE_BUCKETS),
                ("batch_gcups", (ctypes.c_float * TUNE_CANDIDATES) * TUNE_BUCKETS),
                ("rows", ctypes.c_int32 * TUNE_BUCKETS), ("waves", ctypes.c_int32 * TUNE_BUCKETS),
                ("batch_rows", ctypes.c_int32 * TUNE_BUCKETS),
                ("batch_waves", ctypes.c_int32 * TUNE_BUCKETS),
                ("intra_cand_rows", ctypes.c_int32 * TUNE_INTRA_CANDIDATES),
                ("intra_cand_waves", ctypes.c_int32 * TUNE_INTRA_CANDIDATES),
                ("intra_ms", (ctypes.c_float * TUNE_INTRA_CANDIDATES) * TUNE_BUCKETS),
                ("intra_rows", ctypes.c_int32 * TUNE_BUCKETS),
                ("intra_waves", ctypes.c_int32 * TUNE_BUCKETS),
                ("from_cache", ctypes.c_int32)]


# name -> (restype, argtypes); every symbol include/swdb.h declares
P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
SIGNATURES = {
    "sw_db_load": (ctypes.c_int, [P, P, I64, ctypes.POINTER(P)]),
    "sw_db_load_ex": (ctypes.c_int, [P, P, I64, I32, ctypes.POINTER(P)]),
    "sw_db_free": (None, [P]),
    "sw_db_info": (ctypes.c_int, [P, P, P, P, P]),
    "sw_search": (ctypes.c_int, [P, P, I32, P, I32, I32, P]),
    "sw_search_async": (ctypes.c_int, [P, P, I32, P, I32, I32, P, P]),
    "sw_search_async_noalloc": (ctypes.c_int, [P, P, I32, P, I32, I32, P, P]),
    "sw_search_topk": (ctypes.c_int, [P, P, I32, P, I32, I32, I32, P, P]),
    "sw_traceback": (ctypes.c_int, [P, P, I32, P, I32, I32, P, I32, P, P, I64, P]),
    "sw_search_topk_async": (ctypes.c_int, [P, P, I32, P, I32, I32, I32, P, P, P]),
    "sw_search_hybrid": (ctypes.c_int, [P, P, I32, P, I32, I32, I32, P,
                                        ctypes.POINTER(HybridStats)]),
    "sw_host_search": (ctypes.c_int, [P, P, I64, P, I32, P, I32, I32, I32, P]),
    "sw_search_mode": (ctypes.c_int, [P, P, I32, P, I32, I32, I32, P]),
    "sw_search_mode_async": (ctypes.c_int, [P, P, I32, P, I32, I32, I32, P, P]),
    "sw_search_batch": (ctypes.c_int, [P, P, P, I32, P, I32, I32, P]),
    "sw_search_batch_async": (ctypes.c_int, [P, P, P, I32, P, I32, I32, P, P]),
    "sw_last_error": (ctypes.c_char_p, []),
    "sw_set_option": (ctypes.c_int, [P, I32, I64]),
    "sw_get_stats": (ctypes.c_int, [P, ctypes.POINTER(Stats)]),
    "sw_autotune": (ctypes.c_int, [P, ctypes.POINTER(TuneReport)]),
    "sw_autotune_ex": (ctypes.c_int, [P, P, I32, ctypes.c_char_p, ctypes.POINTER(TuneReport)]),
    "sw_plan": (ctypes.c_int, [P, P, I64, I32, ctypes.POINTER(PlanInfo)]),
    "sw_ctx_create": (ctypes.c_int, [P, ctypes.POINTER(P)]),
    "sw_ctx_free": (None, [P]),
    "sw_ctx_bytes": (I64, [P]),
    "sw_ctx_search_async": (ctypes.c_int, [P, P, I32, P, I32, I32, P, P]),
    "sw_ctx_search_batch_async": (ctypes.c_int, [P, P, P, I32, P, I32, I32, P, P]),
    "sw_ctx_set_option": (ctypes.c_int, [P, I32, I64]),
    "sw_ctx_get_stats": (ctypes.c_int, [P, ctypes.POINTER(Stats)]),
    "sw_pack": (ctypes.c_int, [P, P, I64, I32, P, P, P, P]),
}

_lib = None


def lib():
    """Loads libswdb.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libswdb.so is not built (%s); run "
                              "`python -m paper_2203_11100_amd.build`" % LIB_PATH)
        try:
            import torch
            # PyTorch ships its own HIP runtime; it must open the GPU before
            # this library's runtime does, or it finds no device afterwards
            torch.cuda.is_available()
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc != SW_OK:
        msg = lib().sw_last_error()
        raise SwError(rc, msg.decode() if msg else "")
