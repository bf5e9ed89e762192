"""Brute-force k-nearest-neighbour search on AMD Instinct MI355X (gfx950).

Thin Python binding over the C ABI in include/knn.h.  Every step of the
search runs in the library's HIP kernels; this module only checks tensor
arguments, allocates outputs and passes pointers and the current stream.
There is no CPU fallback: without the built library every call raises.

    dist, idx = search(Q, R, k, metric="l2")          # one-shot, float32
    refs = Refs(R, storage="bf16")                     # resident set
    dist, idx = refs.search(Q, k, precision="bf16")    # BF16 MFMA + exact re-rank
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import METRICS, PRECISIONS, KnnError, check, load

__all__ = ["search", "Refs", "KnnError", "METRICS", "PRECISIONS", "load", "timing"]

KERNELS = ("centre", "prep_refs", "prep_queries", "fused_l2_f32", "fused_l2_bf16", "fused_l2_f16",
           "fused_l1_f32", "fused_linf_f32", "finalize")


class timing:
    """Per-kernel HIP-event timing inside the library (knn_timing_*)."""

    @staticmethod
    def enable(on: bool = True):
        check(load().knn_timing_enable(int(on)))

    @staticmethod
    def reset():
        check(load().knn_timing_reset())

    @staticmethod
    def read(name: str):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        check(load().knn_timing_read(name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    @staticmethod
    def all():
        return {k: timing.read(k) for k in KERNELS if timing.read(k)[1] > 0}


def _stream_ptr(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _points(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or x.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if x.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    return x.contiguous()


def _outputs(n: int, k: int, device, out):
    if out is not None:
        dist, idx = out
        if dist.shape != (n, k) or idx.shape != (n, k) or dist.dtype != torch.float32 or idx.dtype != torch.int32:
            raise ValueError("out must be (float32 [n,k], int32 [n,k]) tensors")
        if not (dist.is_contiguous() and idx.is_contiguous()):
            raise ValueError("out tensors must be contiguous")
        return dist, idx
    return (torch.empty((n, k), dtype=torch.float32, device=device),
            torch.empty((n, k), dtype=torch.int32, device=device))


def search(Q: torch.Tensor, R: torch.Tensor, k: int, metric: str = "l2", out=None, stream=None):
    """One-shot float32 brute force (knn_search): returns (dist [n,k], idx [n,k] int32)."""
    lib = load()
    Q = _points(Q, "Q")
    R = _points(R, "R")
    if Q.shape[1] != R.shape[1]:
        raise ValueError("Q and R differ in dimension")
    n, d = Q.shape
    m = R.shape[0]
    dist, idx = _outputs(n, k, Q.device, out)
    check(lib.knn_search(ctypes.c_void_p(Q.data_ptr()), n, ctypes.c_void_p(R.data_ptr()), m, d, int(k),
                         METRICS[metric], ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                         _stream_ptr(stream)))
    return dist, idx


class Refs:
    """A resident reference set (knn_create_refs / knn_search_refs / knn_destroy_refs)."""

    def __init__(self, R: torch.Tensor, storage: str = "fp32", keep_fp32_master: bool = True, stream=None):
        lib = load()
        R = _points(R, "R")
        self.m, self.d = R.shape
        self.storage = storage
        self.device = R.device
        h = ctypes.c_void_p()
        check(lib.knn_create_refs(ctypes.c_void_p(R.data_ptr()), self.m, self.d, PRECISIONS[storage],
                                  int(bool(keep_fp32_master)), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        # the copy is enqueued on the stream; keep R alive until it has run
        (torch.cuda.current_stream() if stream is None else stream).synchronize()

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("reference set already closed")
        return self._h

    def search(self, Q: torch.Tensor, k: int, metric: str = "l2", precision: str | None = None,
               s_extra: int = -1, out=None, stream=None):
        lib = load()
        Q = _points(Q, "Q")
        if Q.shape[1] != self.d:
            raise ValueError("Q has the wrong dimension for this reference set")
        n = Q.shape[0]
        prec = self.storage if precision is None else precision
        dist, idx = _outputs(n, k, Q.device, out)
        check(lib.knn_search_refs(self.handle, ctypes.c_void_p(Q.data_ptr()), n, int(k), METRICS[metric],
                                  PRECISIONS[prec], int(s_extra), ctypes.c_void_p(dist.data_ptr()),
                                  ctypes.c_void_p(idx.data_ptr()), _stream_ptr(stream)))
        return dist, idx

    def close(self):
        if self._h is not None:
            check(load().knn_destroy_refs(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
