"""GPU parity of the per-lane-selection kernels (padded dimension <= 128),
through the C ABI: Manhattan / infinity norm with one query per lane, and
float32 Euclidean on 32x32 MFMA tiles with one query per lane pair.

Every case is checked against the FP64 oracle (relative 1e-5 on distances,
tie-aware indices).  Integer-grid data (all distances exact in float32, many
exact ties) must reproduce the oracle bit for bit, tie order included.  The
same searches through the general kernels (KNN_FUSED_LANE=0) must pass the
same checks, and forced slice counts (KNN_FUSED_P) exercise many short
slices, slices shorter than the list, and a single slice.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
import synthdata
from oracle.check import compare

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def K():
    import torch

    import paper_0804_1448_amd as K

    assert torch.cuda.is_available()
    K.load()
    return K


def banner(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def run(K, Q, R, k, metric, env=None):
    import torch

    saved = {}
    for key, val in (env or {}).items():
        saved[key] = os.environ.get(key)
        os.environ[key] = str(val)
    try:
        dist, idx = K.search(torch.from_numpy(np.ascontiguousarray(Q)).cuda(),
                             torch.from_numpy(np.ascontiguousarray(R)).cuda(), k, metric)
        torch.cuda.synchronize()
    finally:
        for key, val in saved.items():
            if val is None:
                del os.environ[key]
            else:
                os.environ[key] = val
    return dist.cpu().numpy(), idx.cpu().numpy()


def check(Q, R, k, metric, dist, idx):
    rep = compare(Q, R, k, metric, dist, idx, tol=TOL)
    assert rep["ok"], rep
    assert np.all(np.diff(dist, axis=1) >= 0)


# (n, m, d, k, data): one query and one reference; n around multiples of 64;
# every chunk shape of the padded dimension (16 .. 128, full and short last
# 64-dim chunks); k = 1; k' = k + 8 above 64 (two waves per workgroup)
SHAPES = [
    (1, 1, 1, 1, "uniform"), (63, 9, 3, 9, "uniform"), (65, 1000, 16, 20, "gmm"),
    (127, 4099, 17, 20, "uniform"), (128, 3000, 48, 1, "gmm"), (257, 5000, 64, 32, "gmm"),
    (300, 7001, 80, 20, "uniform"), (200, 9000, 96, 20, "gmm"), (70, 6000, 112, 56, "uniform"),
    (190, 12345, 128, 20, "gmm"), (100, 3000, 40, 100, "gmm"),
]


def data(kind, n, m, d, seed):
    if kind == "uniform":
        return synthdata.uniform((n, d), seed, 1), synthdata.uniform((m, d), seed, 0)
    return synthdata.gmm(n, d, 16, 0.05, seed, 1), synthdata.gmm(m, d, 16, 0.05, seed, 0)


@pytest.mark.parametrize("metric", ["l2", "l1", "linf"])
@pytest.mark.parametrize("n,m,d,k,kind", SHAPES)
def test_lane_shapes(K, n, m, d, k, kind, metric):
    banner(f"lane n={n} m={m} d={d} k={k} {kind} {metric}")
    Q, R = data(kind, n, m, d, 700 + n + d + k)
    check(Q, R, k, metric, *run(K, Q, R, k, metric))


@pytest.mark.parametrize("metric", ["l1", "linf"])
def test_lane_integer_grid_is_exact(K, metric):
    """Integers in [0, 5): every distance is an exact float32 integer, so
    the result (ties broken by index) must equal the oracle bit for bit."""
    banner(f"lane integer grid {metric}")
    Q = synthdata.integer_grid((333, 24), 0, 5, 41, 1)
    R = synthdata.integer_grid((7000, 24), 0, 5, 41, 0)
    for P in (0, 1, 37):
        dist, idx = run(K, Q, R, 20, metric, {"KNN_FUSED_P": P} if P else None)
        D, I = oracle.knn(Q, R, 20, metric)
        assert np.array_equal(idx, I.astype(np.int32)), P
        assert np.array_equal(dist, D.astype(np.float32)), P


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("P", [1, 7, 64])
def test_lane_forced_slices(K, P, metric):
    """A single slice, uneven slices, and slices of 32 references (about
    the 28-key lists, which may then never fill)."""
    banner(f"lane P={P} {metric}")
    m = 2000 if P == 64 else 5000
    Q, R = data("gmm", 150, m, 33, 800 + P)
    check(Q, R, 20, metric, *run(K, Q, R, 20, metric, {"KNN_FUSED_P": P}))


def test_lane_k_equals_m_is_a_permutation(K):
    banner("lane k = m")
    Q, R = data("uniform", 70, 120, 10, 91)
    for metric in ("l2", "l1", "linf"):
        dist, idx = run(K, Q, R, 120, metric)
        check(Q, R, 120, metric, dist, idx)
        assert np.all(np.sort(idx, axis=1) == np.arange(120)[None, :])


@pytest.mark.parametrize("metric", ["l2", "l1", "linf"])
def test_lane_and_general_kernels_agree_with_oracle(K, metric):
    banner(f"lane vs general {metric}")
    Q, R = data("gmm", 500, 20000, 96, 92)
    a = run(K, Q, R, 20, metric)
    b = run(K, Q, R, 20, metric, {"KNN_FUSED_LANE": 0})
    check(Q, R, 20, metric, *a)
    check(Q, R, 20, metric, *b)


def test_lane_l2_integer_grid_is_exact(K):
    """Integers in [0, 6) whose first 256 references average exactly 2.5 per
    dimension (rows 128..255 mirror rows 0..127), so the Euclidean centre is
    2.5, every translated value a half-integer, and every score, norm and
    distance exact in float32: the result must equal the oracle bit for bit,
    tie order included."""
    banner("lane l2 integer grid")
    Q = synthdata.integer_grid((333, 40), 0, 6, 42, 1)
    R = synthdata.integer_grid((7000, 40), 0, 6, 42, 0)
    R[128:256] = 5.0 - R[0:128]
    D, I = oracle.knn(Q, R, 20, "l2")
    for P in (0, 1, 37):
        dist, idx = run(K, Q, R, 20, "l2", {"KNN_FUSED_P": P} if P else None)
        assert np.array_equal(idx, I.astype(np.int32)), P
        assert np.array_equal(dist, D.astype(np.float32)), P
