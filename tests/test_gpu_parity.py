"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: relative 1e-5 on distances (float32 path) and tie-aware indices
(a returned index may differ from the oracle's only where another reference
lies within the tolerance at that rank).  Hand-worked cases must match
bit-exactly, tie order included.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import oracle
import synthdata
from oracle.check import compare

pytestmark = pytest.mark.gpu
TOL = 1e-5
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def K():
    import torch

    import paper_0804_1448_amd as K

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    K.load()
    return K


def banner(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_search(K, Q, R, k, metric, refs_storage=None, precision=None, s_extra=-1):
    import torch

    Qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    Rd = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    if refs_storage is None:
        dist, idx = K.search(Qd, Rd, k, metric)
    else:
        refs = K.Refs(Rd, storage=refs_storage)
        dist, idx = refs.search(Qd, k, metric, precision=precision, s_extra=s_extra)
        torch.cuda.synchronize()
        refs.close()
    torch.cuda.synchronize()
    return dist.cpu().numpy(), idx.cpu().numpy()


def make_data(kind, n, m, d, seed):
    if kind == "uniform":
        return synthdata.uniform((n, d), seed, 1), synthdata.uniform((m, d), seed, 0)
    if kind == "gmm":
        return synthdata.gmm(n, d, 16, 0.05, seed, 1), synthdata.gmm(m, d, 16, 0.05, seed, 0)
    if kind == "grid":  # integer coordinates: exact in every precision, many exact ties
        return synthdata.integer_grid((n, d), 0, 5, seed, 1), synthdata.integer_grid((m, d), 0, 5, seed, 0)
    if kind == "dups":  # every reference duplicated
        R = synthdata.uniform(((m + 1) // 2, d), seed, 0)
        return synthdata.uniform((n, d), seed, 1), np.ascontiguousarray(np.repeat(R, 2, axis=0)[:m])
    if kind == "offset":  # large common offset: cancellation in |r|^2 - 2 q.r
        return synthdata.uniform((n, d), seed, 1) + 1000, synthdata.uniform((m, d), seed, 0) + 1000
    raise ValueError(kind)


def assert_parity(Q, R, k, metric, dist, idx, tol=TOL):
    rep = compare(Q, R, k, metric, dist, idx, tol=tol)
    assert rep["ok"], rep
    assert np.all(np.diff(dist, axis=1) >= 0), "distances not ascending"
    return rep


# ------------------------------------------------------------ hand-worked
def test_hand_worked_2d_bit_exact(K):
    g = json.load(open(os.path.join(HERE, "golden", "hand_2d.json")))
    R = np.array(g["R"], dtype=np.float32)
    for c in g["cases"]:
        q = np.array([c["q"]], dtype=np.float32)
        want = (np.sqrt(np.array(c["dist_sq"], np.float32)) if "dist_sq" in c
                else np.array(c["dist"], np.float32))
        for k in range(1, 6):
            banner(f"hand_2d q={c['q']} {c['metric']} k={k}")
            dist, idx = gpu_search(K, q, R, k, c["metric"])
            assert idx[0].tolist() == c["idx"][:k], (c, k, idx)
            assert np.array_equal(dist[0], want[:k]), (c, k, dist)


# ---------------------------------------------------------------- grid
GRID = [
    # (n, m, d, k, data)
    (1, 1, 1, 1, "uniform"), (7, 5, 2, 5, "uniform"), (64, 21, 3, 20, "uniform"),
    (64, 1000, 16, 8, "uniform"), (300, 4097, 17, 20, "gmm"), (33, 4097, 32, 32, "uniform"),
    (129, 1000, 96, 100, "gmm"), (70, 2500, 128, 20, "gmm"), (64, 777, 129, 10, "uniform"),
    (200, 3000, 8, 20, "grid"), (100, 1500, 5, 1, "grid"), (96, 2000, 24, 16, "dups"),
    (80, 1200, 32, 20, "offset"), (5, 300, 12, 300, "uniform"), (40, 65, 7, 64, "gmm"),
    (1, 5000, 64, 100, "uniform"), (513, 64, 3, 7, "grid"),
]


@pytest.mark.parametrize("metric", ["l2", "l1", "linf"])
@pytest.mark.parametrize("n,m,d,k,data", GRID)
def test_grid(K, n, m, d, k, data, metric):
    banner(f"grid n={n} m={m} d={d} k={k} {data} {metric}")
    Q, R = make_data(data, n, m, d, seed=100 + n + m + d)
    dist, idx = gpu_search(K, Q, R, k, metric)
    assert_parity(Q, R, k, metric, dist, idx)


# ------------------------------------------------- named workloads
@pytest.mark.parametrize("metric", ["l2", "l1", "linf"])
def test_uniform4096_d32_full(K, metric):
    banner(f"uniform4096_d32 {metric}")
    R, Q, p = synthdata.workload("uniform4096_d32")
    dist, idx = gpu_search(K, Q, R, p["k"], metric)
    assert_parity(Q, R, p["k"], metric, dist, idx)


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_gmm16384_d96_sampled(K, metric):
    """Full-size workload (the benchmark's launch configuration); oracle on a query sample."""
    import torch

    banner(f"gmm16384_d96 {metric}")
    R, Q, p = synthdata.workload("gmm16384_d96")
    dist, idx = gpu_search(K, Q, R, p["k"], metric)
    rows = np.random.default_rng(5).choice(Q.shape[0], 384, replace=False)
    rep = compare(Q, R, p["k"], metric, dist, idx, tol=TOL, rows=rows)
    assert rep["ok"], rep
    assert np.all(np.diff(dist, axis=1) >= 0)
    # every row: valid, distinct indices
    assert idx.min() >= 0 and idx.max() < R.shape[0]
    s = np.sort(idx, axis=1)
    assert np.all(s[:, 1:] != s[:, :-1])
    del torch


# ---------------------------------------------------------- invariants
def test_power_of_two_scaling_bit_exact(K):
    Q, R = make_data("gmm", 100, 3000, 40, 7)
    for metric in ("l2", "l1", "linf"):
        d1, i1 = gpu_search(K, Q, R, 20, metric)
        d2, i2 = gpu_search(K, Q * 8, R * 8, 20, metric)
        assert np.array_equal(i1, i2) and np.array_equal(d1 * 8, d2), metric


def test_query_independence_bit_exact(K):
    Q, R = make_data("uniform", 600, 5000, 32, 8)
    for metric in ("l2", "l1"):
        d1, i1 = gpu_search(K, Q, R, 20, metric)
        d2, i2 = gpu_search(K, Q[123:130], R, 20, metric)
        assert np.array_equal(i1[123:130], i2) and np.array_equal(d1[123:130], d2)


def test_reference_permutation(K):
    Q, R = make_data("uniform", 64, 2000, 16, 9)
    perm = np.random.default_rng(1).permutation(R.shape[0])
    d1, i1 = gpu_search(K, Q, R, 20, "l2")
    d2, i2 = gpu_search(K, Q, np.ascontiguousarray(R[perm]), 20, "l2")
    assert np.array_equal(perm[i2], i1) and np.array_equal(d1, d2)


def test_prefix_in_k(K):
    Q, R = make_data("gmm", 50, 2000, 20, 10)
    d1, i1 = gpu_search(K, Q, R, 30, "l2")
    d2, i2 = gpu_search(K, Q, R, 12, "l2")
    assert np.array_equal(i1[:, :12], i2) and np.array_equal(d1[:, :12], d2)


def test_k_equals_m_is_permutation(K):
    Q, R = make_data("uniform", 9, 150, 6, 11)
    for metric in ("l2", "l1", "linf"):
        dist, idx = gpu_search(K, Q, R, 150, metric)
        assert np.all(np.sort(idx, axis=1) == np.arange(150))
        assert_parity(Q, R, 150, metric, dist, idx)


def test_deterministic(K):
    Q, R = make_data("gmm", 300, 6000, 48, 12)
    a = gpu_search(K, Q, R, 20, "l2")
    b = gpu_search(K, Q, R, 20, "l2")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------ resident sets and precision
def test_refs_fp32_matches_one_shot(K):
    Q, R = make_data("gmm", 200, 3000, 64, 13)
    for metric in ("l2", "l1", "linf"):
        a = gpu_search(K, Q, R, 20, metric)
        b = gpu_search(K, Q, R, 20, metric, refs_storage="fp32")
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("offset", [0.0, 1000.0])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_low_precision_recall(K, prec, offset):
    banner(f"low precision {prec} offset {offset}")
    Q = synthdata.gmm(512, 128, 64, 0.1, 21, 1) + np.float32(offset)
    R = synthdata.gmm(20000, 128, 64, 0.1, 21, 0) + np.float32(offset)
    dist, idx = gpu_search(K, Q, R, 32, "l2", refs_storage=prec, precision=prec, s_extra=32)
    rep = compare(Q, R, 32, "l2", dist, idx, tol=TOL)
    assert rep["bad_index_rows"] == 0
    assert rep["recall"] >= 0.999, rep
    assert rep["max_rel_err_hits"] <= TOL and rep["bad_pair"] == 0 and rep["bad_index_rows"] == 0, rep
    assert np.all(np.diff(dist, axis=1) >= 0)


def test_errors_leave_outputs_untouched(K):
    import torch

    Q = torch.rand(4, 3, device="cuda")
    R = torch.rand(10, 3, device="cuda")
    dist = torch.full((4, 11), -7.0, device="cuda")
    idx = torch.full((4, 11), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KnnError):
        K.search(Q, R, 11, "l2", out=(dist, idx))
    torch.cuda.synchronize()
    assert bool((dist == -7).all()) and bool((idx == -7).all())
    refs = K.Refs(R, storage="fp32")
    with pytest.raises(K.KnnError):
        refs.search(Q, 2, "l2", precision="bf16")
    refs.close()
    refs16 = K.Refs(R, storage="bf16")
    with pytest.raises(K.KnnError):
        refs16.search(Q, 2, "l1", precision="bf16")
    refs16.close()


@pytest.mark.parametrize("metric,storage,prec,k", [("l2", None, None, 20), ("l1", None, None, 20),
                                                   ("linf", None, None, 5), ("l2", "bf16", "bf16", 32),
                                                   ("l2", "fp16", "fp16", 50)])
def test_many_slices_merged_first(K, metric, storage, prec, k):
    """A few queries against many references: the search spreads over more
    slices than the finalize merges at once (up to 256), so the slice lists
    are merged in groups first.  The result must match the oracle and equal,
    bit for bit, the search with at most 64 slices (KNN_FUSED_P=16), whose
    lists the finalize merges directly: the kept top-k' under the (score,
    index) order does not depend on the slicing."""
    n, m, d = 37, 400000, 48
    banner(f"many slices {metric} {prec} k={k}: n={n} m={m} d={d}")
    Q, R = make_data("gmm", n, m, d, 4242)
    a = gpu_search(K, Q, R, k, metric, refs_storage=storage, precision=prec)
    os.environ["KNN_FUSED_P"] = "16"
    try:
        b = gpu_search(K, Q, R, k, metric, refs_storage=storage, precision=prec)
    finally:
        del os.environ["KNN_FUSED_P"]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    rep = compare(Q, R, k, metric, a[0], a[1], tol=TOL)
    if prec is None:
        assert rep["ok"], rep
    else:
        assert rep["bad_index_rows"] == 0 and rep["bad_pair"] == 0 and rep["recall"] >= 0.999, rep


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_k_at_the_limit_and_above(K, metric):
    """k = 440 (k' = 448, the most candidates the fused kernels keep) matches
    the oracle; k = 441 is rejected as unsupported with the outputs untouched."""
    import torch

    banner(f"k limit {metric}")
    Q, R = make_data("uniform", 100, 6000, 24, 4401)
    dist, idx = gpu_search(K, Q, R, 440, metric)
    assert_parity(Q, R, 440, metric, dist, idx)
    Qd, Rd = torch.from_numpy(Q).cuda(), torch.from_numpy(R).cuda()
    out = (torch.full((100, 441), -5.0, device="cuda"), torch.full((100, 441), -5, dtype=torch.int32, device="cuda"))
    with pytest.raises(K.KnnError) as e:
        K.search(Qd, Rd, 441, metric, out=out)
    assert e.value.status == -2
    torch.cuda.synchronize()
    assert bool((out[0] == -5.0).all()) and bool((out[1] == -5).all())
