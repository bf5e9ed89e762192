"""GPU parity of the 16-bit Euclidean kernel with 32x32 tiles and
register-resident lists (k' <= 64, d <= 128), through the C ABI.

Every case is checked against the FP64 oracle: indices tie-aware, distances
of the returned hits within 1e-5 after the exact float32 re-rank, recall@k
of the low-precision candidate selection >= 0.999.  Integer-grid data (exact
in both 16-bit formats, all scores exact, many exact ties) must reproduce the
oracle bit for bit, tie order included.  The same inputs through the general
kernel (KNN_FUSED_WIDE=0) must pass the same checks.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import synthdata
from oracle.check import compare
import oracle

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


def search16(K, Q, R, k, prec, s_extra=32):
    import torch

    refs = K.Refs(torch.from_numpy(np.ascontiguousarray(R)).cuda(), storage=prec)
    dist, idx = refs.search(torch.from_numpy(np.ascontiguousarray(Q)).cuda(), k, "l2", precision=prec,
                            s_extra=s_extra)
    torch.cuda.synchronize()
    out = dist.cpu().numpy(), idx.cpu().numpy()
    refs.close()
    return out


def check(Q, R, k, dist, idx, min_recall=0.999):
    rep = compare(Q, R, k, "l2", dist, idx, tol=TOL)
    assert rep["bad_index_rows"] == 0, rep
    assert rep["recall"] >= min_recall, rep
    assert rep["max_rel_err_hits"] <= TOL and rep["bad_pair"] == 0 and rep["bad_index_rows"] == 0, rep
    assert np.all(np.diff(dist, axis=1) >= 0)
    return rep


# (n, m, d, k, precision, data): tiny sets, ragged n and m, every padded
# width (32, 64, 96, 128), many slices (small n, large m), k = 1
SHAPES = [
    (1, 50, 16, 1, "bf16", "uniform"),
    (17, 130, 32, 10, "fp16", "uniform"),
    (255, 1000, 48, 32, "bf16", "gmm"),
    (257, 4097, 64, 20, "fp16", "gmm"),
    (600, 20000, 96, 32, "bf16", "gmm"),
    (300, 9000, 128, 32, "fp16", "gmm"),
    (64, 70000, 100, 32, "bf16", "gmm"),
    (3000, 3000, 128, 1, "bf16", "gmm"),
    (513, 12345, 80, 7, "fp16", "uniform"),
]


def data(kind, n, m, d, seed):
    if kind == "uniform":
        return synthdata.uniform((n, d), seed, 1), synthdata.uniform((m, d), seed, 0)
    return synthdata.gmm(n, d, 32, 0.08, seed, 1), synthdata.gmm(m, d, 32, 0.08, seed, 0)


@pytest.mark.parametrize("n,m,d,k,prec,kind", SHAPES)
def test_wide_shapes(K, n, m, d, k, prec, kind):
    banner(f"wide n={n} m={m} d={d} k={k} {prec} {kind}")
    Q, R = data(kind, n, m, d, 300 + d + k)
    dist, idx = search16(K, Q, R, k, prec)
    check(Q, R, k, dist, idx)


def test_wide_k_equals_m_is_a_permutation(K):
    banner("wide k = m")
    Q, R = data("uniform", 40, 40, 24, 77)
    dist, idx = search16(K, Q, R, 40, "fp16")
    check(Q, R, 40, dist, idx, min_recall=1.0)
    assert np.all(np.sort(idx, axis=1) == np.arange(40)[None, :])


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_wide_integer_grid_is_exact(K, prec):
    """Integers in [0, 6) whose first 256 references average exactly 2.5 per
    dimension (rows 128..255 mirror rows 0..127), so the Euclidean centre is
    2.5 and every translated value is a half-integer: rows, half-norms and
    scores are exact in both 16-bit formats and in float32, and the kept
    candidates and the re-ranked result must equal the oracle bit for bit,
    tie order included."""
    banner(f"wide integer grid {prec}")
    Q = synthdata.integer_grid((700, 64), 0, 6, 88, 1)
    R = synthdata.integer_grid((9000, 64), 0, 6, 88, 0)
    R[128:256] = 5.0 - R[0:128]
    k = 32
    dist, idx = search16(K, Q, R, k, prec)
    D, I = oracle.knn(Q, R, k, "l2")
    assert np.array_equal(idx, I.astype(np.int32))
    assert np.array_equal(dist, D.astype(np.float32))


def test_wide_and_general_kernels_agree_with_oracle(K):
    banner("wide vs general")
    Q, R = data("gmm", 400, 30000, 128, 91)
    k = 32
    a = search16(K, Q, R, k, "bf16")
    os.environ["KNN_FUSED_WIDE"] = "0"
    try:
        b = search16(K, Q, R, k, "bf16")
    finally:
        del os.environ["KNN_FUSED_WIDE"]
    ra = check(Q, R, k, *a)
    rb = check(Q, R, k, *b)
    # the two kernels sum the 16-bit products in different orders; their
    # results may differ only where the oracle allows it
    assert abs(ra["recall"] - rb["recall"]) <= 0.002


@pytest.mark.parametrize("n,m,d,k", [(4096, 262144, 64, 20), (100, 1048576, 32, 20), (64, 600000, 100, 56),
                                     (700, 9000, 96, 20)])
def test_wide_fp32_matches_oracle_and_general(K, n, m, d, k):
    """Float32 Euclidean (k + 8 <= 64, d <= 128).  Resident set with the lane
    kernels switched off (KNN_FUSED_LANE=0): slices of at least 16384
    references run the 32x32-tile kernel, shorter ones the general kernel.
    Resident set by default: the 32x32-tile kernel from 16384, the lane kernel
    (row-major rows) below.  One-shot search: the lane kernel on tiled rows up
    to slices of 131072, then the 32x32-tile kernel.  All three must pass the
    same oracle check (on a query sample for the larger cases)."""
    import torch

    banner(f"wide fp32 n={n} m={m} d={d} k={k}")
    Q = synthdata.gmm(n, d, 64, 0.08, 500 + d + k, 1)
    R = synthdata.gmm(m, d, 64, 0.08, 500 + d + k, 0, threads=8)
    Qd, Rd = torch.from_numpy(Q).cuda(), torch.from_numpy(R).cuda()
    refs = K.Refs(Rd, storage="fp32")

    def resident():
        out = [t.cpu().numpy() for t in refs.search(Qd, k, "l2")]
        torch.cuda.synchronize()
        return out

    os.environ["KNN_FUSED_LANE"] = "0"
    try:
        a = resident()
    finally:
        del os.environ["KNN_FUSED_LANE"]
    b = resident()
    c = [t.cpu().numpy() for t in K.search(Qd, Rd, k, "l2")]
    refs.close()
    rows = np.arange(n) if n * m <= 2e8 else np.random.default_rng(5).choice(n, 48, replace=False)
    ref = oracle.knn(Q[rows], R, k, "l2")
    for dist, idx in (a, b, c):
        rep = compare(Q, R, k, "l2", dist, idx, tol=TOL, ref=ref, rows=rows)
        assert rep["ok"], rep


# k' = k + s in (64, 128]: two list keys per lane
SHAPES_TWO_KEYS = [
    (129, 3000, 64, 50, 32, "fp16", "gmm"),       # k' = 82
    (300, 20000, 128, 96, 32, "bf16", "gmm"),     # k' = 128
    (70, 50000, 32, 100, 28, "fp16", "uniform"),  # k' = 128
    (257, 1000, 96, 65, 1, "bf16", "uniform"),    # k' = 66
    (33, 100, 16, 80, 32, "fp16", "uniform"),     # k' = 100 of m = 100
]


@pytest.mark.parametrize("n,m,d,k,s,prec,kind", SHAPES_TWO_KEYS)
def test_wide_two_keys_per_lane(K, n, m, d, k, s, prec, kind):
    banner(f"wide two keys n={n} m={m} d={d} k={k} s={s} {prec} {kind}")
    Q, R = data(kind, n, m, d, 500 + d + k)
    dist, idx = search16(K, Q, R, k, prec, s_extra=s)
    check(Q, R, k, dist, idx)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_wide_two_keys_integer_grid_is_exact(K, prec):
    """The integer-grid case of test_wide_integer_grid_is_exact with k' = 128
    (k = 96): the two-register lists must reproduce the oracle bit for bit."""
    banner(f"wide two keys integer grid {prec}")
    Q = synthdata.integer_grid((300, 64), 0, 6, 89, 1)
    R = synthdata.integer_grid((9000, 64), 0, 6, 89, 0)
    R[128:256] = 5.0 - R[0:128]
    k = 96
    dist, idx = search16(K, Q, R, k, prec, s_extra=32)
    D, I = oracle.knn(Q, R, k, "l2")
    assert np.array_equal(idx, I.astype(np.int32))
    assert np.array_equal(dist, D.astype(np.float32))


@pytest.mark.parametrize("prec,k", [("bf16", 32), ("fp16", 32), ("bf16", 90)])
def test_wide_slices_sharing_a_bound_equal_one_slice(K, prec, k):
    """Slices of one query publish their k'-th best and filter with the
    smallest any of them has published; from 8 slices on they also publish
    their r-th best (r = ceil(k' / P)) and filter with the smallest, over
    groups of ceil(k' / r) slices, of the largest value in a group.  Both
    bounds drop only candidates that cannot be among the query's k' best of
    the whole set, so any number of slices (KNN_FUSED_P; the last slice
    shorter), with or without the rank bound (KNN_RANK_SHARE=0), must give
    bitwise the same result as one slice.  k = 90 (k' = 122) takes two list
    keys per lane, and at most 2048 / k' = 16 slices."""
    banner(f"wide shared bound {prec} k={k}")
    Q, R = data("gmm", 300, 200000, 64, 811)
    out = {}
    runs = [(1, "1"), (4, "1"), (8, "1"), (16, "1"), (64, "1"), (64, "0"), (256, "1")]
    for P, rank in runs:
        os.environ["KNN_FUSED_P"] = str(P)
        os.environ["KNN_RANK_SHARE"] = rank
        try:
            out[(P, rank)] = search16(K, Q, R, k, prec)
        finally:
            del os.environ["KNN_FUSED_P"]
            del os.environ["KNN_RANK_SHARE"]
    check(Q, R, k, *out[(1, "1")])
    for key in runs[1:]:
        assert np.array_equal(out[key][1], out[(1, "1")][1]), f"indices differ with {key[0]} slices (rank {key[1]})"
        assert np.array_equal(out[key][0].view(np.uint32), out[(1, "1")][0].view(np.uint32)), \
            f"distances differ with {key[0]} slices (rank {key[1]})"


@pytest.mark.parametrize("n", [1, 33, 224])
def test_wide_small_search_with_empty_waves(K, n):
    """A search of fewer than 256 queries fills one query block only in part.
    From 8 slices on (the kernels with rank slots) a wave whose 32 rows all
    lie past n only copies tiles and takes the barriers: n = 1 leaves seven
    such waves, n = 33 six, n = 224 one (the last).  The live rows must match
    the oracle and, bitwise, the one-slice search, which has no such path."""
    banner(f"wide small search n={n}")
    Q, R = data("gmm", n, 100000, 64, 907)
    out = {}
    for P in (1, 16, 64):
        os.environ["KNN_FUSED_P"] = str(P)
        try:
            out[P] = search16(K, Q, R, 32, "fp16")
        finally:
            del os.environ["KNN_FUSED_P"]
    check(Q, R, 32, *out[1])
    for P in (16, 64):
        assert np.array_equal(out[P][1], out[1][1]), f"indices differ with {P} slices"
        assert np.array_equal(out[P][0].view(np.uint32), out[1][0].view(np.uint32)), f"distances differ with {P} slices"
