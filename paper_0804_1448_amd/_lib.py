"""ctypes loader for ``libknn.so`` (the C ABI declared in include/knn.h)."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# KNN_LIB_PATH selects another build of the same library (the host-sanitizer
# build the CPU tests load); the default is the in-tree libknn.so
LIB_PATH = os.environ.get("KNN_LIB_PATH") or os.path.join(PKG, "libknn.so")

KNN_OK = 0
STATUS = {0: "OK", -1: "INVALID", -2: "UNSUPPORTED", -3: "OOM", -4: "DEVICE", -5: "BUSY", -6: "CANCELLED"}
METRICS = {"l2": 0, "l1": 1, "linf": 2}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}

# name -> (restype, argtypes); every symbol include/knn.h declares
_c = ctypes
SIGNATURES = {
    "knn_version": (_c.c_int, []),
    "knn_last_error": (_c.c_char_p, []),
    "knn_search": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_int32,
                              _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "knn_search_noalloc": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_int32,
                                      _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "knn_search_mahalanobis": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_void_p,
                                          _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "knn_classify": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_void_p,
                                _c.c_int32, _c.c_void_p, _c.c_void_p]),
    "knn_entropy": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p]),
    "knn_create_refs": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p,
                                   _c.POINTER(_c.c_void_p)]),
    "knn_destroy_refs": (_c.c_int, [_c.c_void_p]),
    "knn_refs_info": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int32),
                                 _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "knn_search_refs": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_int32, _c.c_int32,
                                   _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "knn_batch_create": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_int32,
                                    _c.POINTER(_c.c_void_p)]),
    "knn_batch_run": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p]),
    "knn_batch_destroy": (_c.c_int, [_c.c_void_p]),
    "knn_search_batched": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p]),
    "knn_timing_enable": (_c.c_int, [_c.c_int32]),
    "knn_timing_read": (_c.c_int, [_c.c_char_p, _c.POINTER(_c.c_double), _c.POINTER(_c.c_int64)]),
    "knn_timing_reset": (_c.c_int, []),
    "knn_server_create": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.POINTER(_c.c_void_p)]),
    "knn_server_submit": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_void_p,
                                     _c.c_void_p, _c.POINTER(_c.c_uint64)]),
    "knn_server_poll": (_c.c_int, [_c.c_void_p, _c.c_uint64, _c.POINTER(_c.c_int32), _c.POINTER(_c.c_double)]),
    "knn_server_wait": (_c.c_int, [_c.c_void_p, _c.c_uint64, _c.POINTER(_c.c_double)]),
    "knn_server_cancel": (_c.c_int, [_c.c_void_p, _c.c_uint64]),
    "knn_server_stats": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "knn_server_destroy": (_c.c_int, [_c.c_void_p]),
}


class Problem(_c.Structure):
    """knn_problem_t: one instance of a batched search."""

    _fields_ = [("refs", _c.c_void_p), ("Q", _c.c_void_p), ("n", _c.c_int64), ("k", _c.c_int32),
                ("metric", _c.c_int32), ("dist", _c.c_void_p), ("idx", _c.c_void_p)]


class ServerConfig(_c.Structure):
    """knn_server_config_t."""

    _fields_ = [("mem_budget", _c.c_int64), ("max_batches", _c.c_int32), ("max_queue", _c.c_int32),
                ("max_batch_queries", _c.c_int32), ("precision", _c.c_int32), ("s_extra", _c.c_int32),
                ("flags", _c.c_int32), ("dry_m", _c.c_int64), ("dry_d", _c.c_int32),
                ("dry_us_per_query", _c.c_double)]


class ServerStats(_c.Structure):
    """knn_server_stats_t."""

    _fields_ = [("submitted", _c.c_int64), ("completed", _c.c_int64), ("rejected_busy", _c.c_int64),
                ("batches", _c.c_int64), ("queries", _c.c_int64), ("peak_batches_in_flight", _c.c_int32),
                ("peak_mem_in_flight", _c.c_int64), ("mem_budget", _c.c_int64), ("cancelled", _c.c_int64)]


KNN_ERR_BUSY = -5
KNN_ERR_CANCELLED = -6
KNN_SERVER_DRY_RUN = 1
KNN_SERVER_ONE_SET = 2


class KnnError(RuntimeError):
    """A non-OK status from the library, with its message."""

    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load the built library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0804_1448_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int) -> None:
    if status != KNN_OK:
        msg = load().knn_last_error().decode(errors="replace")
        raise KnnError(status, msg)
