"""FP64 brute-force k-NN oracle (plain C, loaded with ctypes).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline use it to check the GPU library; the library itself never imports,
loads or calls anything here.  It computes the brute-force method of the
paper's Section 2.1 (all distances in double precision, sort by
(distance, index), keep k) -- see ``knn_oracle.c`` for the exact steps and the
readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_oracle.c")
_LIB = os.path.join(_HERE, "libknn_oracle.so")

METRICS = {"l2": 0, "l1": 1, "linf": 2}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 -fopenmp (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.knn_oracle.restype = ctypes.c_int
        lib.knn_oracle.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        lib.knn_oracle_pairs.restype = ctypes.c_int
        lib.knn_oracle_pairs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        _lib = lib
    return _lib


def _f32(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.float32:
        raise TypeError("oracle inputs are float32 arrays (upcast exactly inside)")
    return a


def knn(Q, R, k: int, metric: str = "l2", mode: str = "select", threads: int = 0):
    """Return (dist float64 [n,k], idx int64 [n,k]) for every query.

    ``mode="sort"`` sorts all m pairs per query (the literal method);
    ``mode="select"`` keeps a k-element heap and sorts it.  Both give the same
    result because (distance, index) is a total order.
    """
    Q = _f32(Q)
    R = _f32(R)
    n, d = Q.shape
    m, d2 = R.shape
    if d != d2:
        raise ValueError("Q and R differ in dimension")
    dist = np.empty((n, k), dtype=np.float64)
    idx = np.empty((n, k), dtype=np.int64)
    rc = _load().knn_oracle(Q.ctypes.data, n, R.ctypes.data, m, d, k, METRICS[metric],
                            {"sort": 0, "select": 1}[mode], int(threads),
                            dist.ctypes.data, idx.ctypes.data)
    if rc != 0:
        raise ValueError(f"knn_oracle rejected the arguments (rc={rc})")
    return dist, idx


def pair_dist(Q, R, qi, rj, metric: str = "l2", threads: int = 0) -> np.ndarray:
    """Double-precision distance of the pairs (Q[qi[c]], R[rj[c]])."""
    Q = _f32(Q)
    R = _f32(R)
    qi = np.ascontiguousarray(qi, dtype=np.int64).ravel()
    rj = np.ascontiguousarray(rj, dtype=np.int64).ravel()
    if qi.shape != rj.shape:
        raise ValueError("qi and rj differ in length")
    if qi.size and (qi.min() < 0 or qi.max() >= Q.shape[0] or rj.min() < 0 or rj.max() >= R.shape[0]):
        raise IndexError("pair index out of range")
    out = np.empty(qi.size, dtype=np.float64)
    rc = _load().knn_oracle_pairs(Q.ctypes.data, R.ctypes.data, Q.shape[1], METRICS[metric],
                                  qi.ctypes.data, rj.ctypes.data, qi.size, out.ctypes.data)
    if rc != 0:
        raise ValueError("knn_oracle_pairs rejected the arguments")
    return out
