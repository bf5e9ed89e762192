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

from ._lib import (KNN_ERR_BUSY, KNN_SERVER_DRY_RUN, KNN_SERVER_ONE_SET, METRICS, PRECISIONS, KnnError, Problem, ServerConfig,
                   ServerStats, check, load)

__all__ = ["search", "search_noalloc", "search_mahalanobis", "classify", "entropy", "Refs", "Batch", "search_batched", "Server", "KnnError", "METRICS", "PRECISIONS", "load",
           "timing"]

KERNELS = ("centre", "prep_refs", "prep_queries", "fused_l2_f32", "fused_l2_bf16", "fused_l2_f16",
           "fused_l1_f32", "fused_linf_f32", "merge", "finalize", "batch_graph")


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


def search_noalloc(Q: torch.Tensor, R: torch.Tensor, k: int, metric: str = "l2", out=None, stream=None):
    """knn_search with the library's fixed device workspace (knn_search_noalloc):
    the library allocates nothing; pass ``out=(dist, idx)`` to allocate nothing here either."""
    lib = load()
    Q = _points(Q, "Q")
    R = _points(R, "R")
    if Q.shape[1] != R.shape[1]:
        raise ValueError("Q and R differ in dimension")
    n, d = Q.shape
    m = R.shape[0]
    dist, idx = _outputs(n, k, Q.device, out)
    check(lib.knn_search_noalloc(ctypes.c_void_p(Q.data_ptr()), n, ctypes.c_void_p(R.data_ptr()), m, d, int(k),
                                 METRICS[metric], ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                 _stream_ptr(stream)))
    return dist, idx


def search_mahalanobis(Q: torch.Tensor, R: torch.Tensor, L: torch.Tensor, k: int, out=None, stream=None):
    """Brute force under d_M(q, r) = ||L^T (q - r)|| (knn_search_mahalanobis),
    L [d, d] float32 on the device with Sigma^-1 = L L^T."""
    lib = load()
    Q = _points(Q, "Q")
    R = _points(R, "R")
    L = _points(L, "L")
    n, d = Q.shape
    m = R.shape[0]
    if R.shape[1] != d or tuple(L.shape) != (d, d):
        raise ValueError("Q [n,d], R [m,d] and L [d,d] required")
    dist, idx = _outputs(n, k, Q.device, out)
    check(lib.knn_search_mahalanobis(ctypes.c_void_p(Q.data_ptr()), n, ctypes.c_void_p(R.data_ptr()), m, d,
                                     ctypes.c_void_p(L.data_ptr()), int(k), ctypes.c_void_p(dist.data_ptr()),
                                     ctypes.c_void_p(idx.data_ptr()), _stream_ptr(stream)))
    return dist, idx


def classify(Q: torch.Tensor, R: torch.Tensor, labels: torch.Tensor, k: int, stream=None) -> torch.Tensor:
    """Majority class of each query's k nearest references (knn_classify);
    labels: int32 [m] on the device.  Returns int32 [n]."""
    lib = load()
    Q = _points(Q, "Q")
    R = _points(R, "R")
    if Q.shape[1] != R.shape[1]:
        raise ValueError("Q and R differ in dimension")
    if labels.dtype != torch.int32 or labels.dim() != 1 or labels.shape[0] != R.shape[0] or labels.device.type != "cuda":
        raise ValueError("labels must be an int32 [m] tensor on the GPU")
    labels = labels.contiguous()
    n, d = Q.shape
    out = torch.empty(n, dtype=torch.int32, device=Q.device)
    check(lib.knn_classify(ctypes.c_void_p(Q.data_ptr()), n, ctypes.c_void_p(R.data_ptr()), R.shape[0], d,
                           ctypes.c_void_p(labels.data_ptr()), int(k), ctypes.c_void_p(out.data_ptr()),
                           _stream_ptr(stream)))
    return out


def entropy(Y: torch.Tensor, k: int, stream=None) -> float:
    """k-NN entropy estimate of the points Y [n, d] in nats (knn_entropy):
    (1/n) sum_i [d log rho_k(y_i) + log(n - 1)] + log c_1(d) - Psi(k)."""
    lib = load()
    Y = _points(Y, "Y")
    n, d = Y.shape
    out = torch.empty(1, dtype=torch.float64, device=Y.device)
    check(lib.knn_entropy(ctypes.c_void_p(Y.data_ptr()), n, d, int(k), ctypes.c_void_p(out.data_ptr()),
                          _stream_ptr(stream)))
    return float(out.item())


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


class Batch:
    """A batched search (knn_batch_*): many (refs, Q, k, metric) instances in a few launches.

    ``problems`` is a list of ``(refs, Q, k, metric)``; outputs are allocated
    here and returned by :meth:`results`.  ``run(use_graph=True)`` captures
    the launch sequence into a HIP graph on its first call and replays it.
    """

    def __init__(self, problems, precision: str = "fp32", s_extra: int = -1, tune: bool = False):
        lib = load()
        self._keep = []
        self._out = []
        arr = (Problem * max(1, len(problems)))()
        for i, (refs, Q, k, metric) in enumerate(problems):
            Q = _points(Q, "Q")
            if Q.shape[1] != refs.d:
                raise ValueError(f"instance {i}: Q has the wrong dimension for its reference set")
            dist, idx = _outputs(Q.shape[0], k, Q.device, None)
            self._keep.append((refs, Q))
            self._out.append((dist, idx))
            arr[i] = Problem(refs.handle.value, Q.data_ptr(), Q.shape[0], int(k), METRICS[metric],
                             dist.data_ptr(), idx.data_ptr())
        h = ctypes.c_void_p()
        check(lib.knn_batch_create(arr, len(problems), PRECISIONS[precision], int(s_extra), 1 if tune else 0,
                                   ctypes.byref(h)))
        self._h = h

    def run(self, use_graph: bool = False, stream=None):
        if self._h is None:
            raise ValueError("batch already closed")
        check(load().knn_batch_run(self._h, int(bool(use_graph)), _stream_ptr(stream)))
        return self

    def results(self):
        return list(self._out)

    def close(self):
        if self._h is not None:
            check(load().knn_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def search_batched(problems, precision: str = "fp32", s_extra: int = -1, stream=None):
    """One-shot batched search: returns [(dist, idx)] in the order of ``problems``."""
    b = Batch(problems, precision, s_extra)
    b.run(False, stream)
    out = b.results()
    (torch.cuda.current_stream() if stream is None else stream).synchronize()
    b.close()
    return out


class Server:
    """Serving engine (knn_server_*): Euclidean requests from host memory,
    continuously batched onto resident reference sets.

    ``sets`` is a list of :class:`Refs` stored in ``precision``.  :meth:`submit` takes a float32 ``(n, d)`` numpy array
    and returns a ticket; :meth:`wait` returns ``(dist, idx, latency_us)`` as
    numpy arrays.  ``submit`` raises :class:`KnnError` with status BUSY when
    ``max_queue`` requests are already waiting.
    """

    def __init__(self, sets, mem_budget: int, max_batches: int = 4, max_queue: int = 1024,
                 max_batch_queries: int = 4096, precision: str = "fp32", s_extra: int = -1, one_set: bool = False):
        import numpy as np

        self._np = np
        lib = load()
        self._sets = list(sets)
        if not self._sets:
            raise ValueError("at least one reference set is required")
        self.d = self._sets[0].d
        cfg = ServerConfig(int(mem_budget), int(max_batches), int(max_queue), int(max_batch_queries),
                           PRECISIONS[precision], int(s_extra), KNN_SERVER_ONE_SET if one_set else 0, 0, 0, 0.0)
        arr = (ctypes.c_void_p * len(self._sets))(*[r.handle.value for r in self._sets])
        h = ctypes.c_void_p()
        check(lib.knn_server_create(arr, len(self._sets), ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._live = {}

    @classmethod
    def dry(cls, nsets: int, m: int, d: int, us_per_query: float, **kw):
        """A server that does no device work (scheduler tests, capacity planning)."""
        srv = cls.__new__(cls)
        import numpy as np

        srv._np = np
        lib = load()
        cfg = ServerConfig(int(kw.get("mem_budget", 1 << 30)), int(kw.get("max_batches", 4)),
                           int(kw.get("max_queue", 1024)), int(kw.get("max_batch_queries", 4096)),
                           PRECISIONS[kw.get("precision", "fp32")], int(kw.get("s_extra", -1)),
                           KNN_SERVER_DRY_RUN | (KNN_SERVER_ONE_SET if kw.get("one_set") else 0),
                           int(m), int(d), float(us_per_query))
        h = ctypes.c_void_p()
        check(lib.knn_server_create(None, int(nsets), ctypes.byref(cfg), ctypes.byref(h)))
        srv._h, srv._live, srv._sets, srv.d = h, {}, [], d
        return srv

    def submit(self, set_index: int, Q, k: int) -> int:
        np = self._np
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        if Q.ndim != 2 or Q.shape[1] != self.d:
            raise ValueError(f"Q must be (n, {self.d})")
        n = Q.shape[0]
        dist = np.empty((n, k), np.float32)
        idx = np.empty((n, k), np.int32)
        t = ctypes.c_uint64()
        check(load().knn_server_submit(self._h, int(set_index), Q.ctypes.data, n, int(k), dist.ctypes.data,
                                       idx.ctypes.data, ctypes.byref(t)))
        self._live[t.value] = (Q, dist, idx)
        return t.value

    def poll(self, ticket: int):
        """``None`` while the request runs, else ``(dist, idx, latency_us)``."""
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        st = load().knn_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(lat))
        if st != 0:
            self._live.pop(ticket, None)
            check(st)
        if not done.value:
            return None
        _, dist, idx = self._live.pop(ticket)
        return dist, idx, lat.value

    def cancel(self, ticket: int) -> bool:
        """Withdraw a request that is still waiting (True); False when it is
        already on the device or complete (it then completes normally)."""
        st = load().knn_server_cancel(self._h, ctypes.c_uint64(ticket))
        if st == KNN_ERR_BUSY:
            return False
        check(st)
        return True

    def wait(self, ticket: int):
        lat = ctypes.c_double()
        st = load().knn_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(lat))
        entry = self._live.pop(ticket, None)
        check(st)
        _, dist, idx = entry
        return dist, idx, lat.value

    def stats(self) -> dict:
        out = ServerStats()
        check(load().knn_server_stats(self._h, ctypes.byref(out)))
        return {name: getattr(out, name) for name, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            check(load().knn_server_destroy(self._h))
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
