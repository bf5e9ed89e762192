"""Pins for the FP64 oracle: checks that do not trust the oracle's own code.

Each pin fixes the oracle against something else the paper or mathematics
determines: hand-worked 2-D cases of the Section 2.1 definition, an exact
rational brute force, a library reduction (scipy distances + stable argsort),
an independent 1-D two-pointer algorithm, invariants of the definition, and the
closed-form rounding bound of the float32 difference form.  The last test
plants mistakes in copies of the oracle source and checks that the pins catch
each of them.
"""
from __future__ import annotations

import json
import math
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synthdata

HERE = os.path.dirname(os.path.abspath(__file__))
METRICS = ["l2", "l1", "linf"]


# ---------------------------------------------------------------- hand-worked
def _golden():
    with open(os.path.join(HERE, "golden", "hand_2d.json")) as f:
        return json.load(f)


def hand_2d_failures(knn_fn):
    """Number of mismatches of ``knn_fn`` against the hand-worked 2-D cases."""
    g = _golden()
    R = np.array(g["R"], dtype=np.float32)
    bad = 0
    for c in g["cases"]:
        q = np.array([c["q"]], dtype=np.float32)
        want = np.sqrt(np.array(c["dist_sq"], float)) if "dist_sq" in c else np.array(c["dist"], float)
        for k in range(1, len(R) + 1):
            d, i = knn_fn(q, R, k, c["metric"])
            bad += int(not np.array_equal(i[0], c["idx"][:k]))
            bad += int(not np.array_equal(d[0], want[:k]))
    return bad


@pytest.mark.parametrize("mode", ["sort", "select"])
def test_hand_worked_2d(mode):
    assert hand_2d_failures(lambda q, R, k, mt: oracle.knn(q, R, k, mt, mode=mode)) == 0


# ------------------------------------------------------------- exact rational
def exact_knn(Q, R, k, metric):
    """Brute force in exact rationals: (squared L2 | L1 | Linf) then (value, index) order."""
    out_v, out_i = [], []
    for q in Q:
        vals = []
        for j, r in enumerate(R):
            diffs = [Fraction(float(a)) - Fraction(float(b)) for a, b in zip(q, r)]
            if metric == "l2":
                v = sum(x * x for x in diffs)
            elif metric == "l1":
                v = sum(abs(x) for x in diffs)
            else:
                v = max(abs(x) for x in diffs)
            vals.append((v, j))
        vals.sort()
        out_v.append([v for v, _ in vals[:k]])
        out_i.append([j for _, j in vals[:k]])
    return out_v, out_i


def exact_failures(knn_fn, trials=60, seed=0):
    rng = np.random.default_rng(seed)
    bad = 0
    for t in range(trials):
        n = int(rng.integers(1, 8))
        m = int(rng.integers(1, 21))
        d = int(rng.integers(1, 6))
        k = int(rng.integers(1, m + 1))
        metric = METRICS[t % 3]
        # dyadic grid with 4 fractional bits: double arithmetic on it is exact
        Q = synthdata.dyadic((n, d), 4, 1000 + t, synthdata.ROLE_QUERIES)
        R = synthdata.dyadic((m, d), 4, 1000 + t, synthdata.ROLE_REFS)
        if t % 4 == 0:  # force duplicates and exact ties
            R = np.round(R)
            Q = np.round(Q)
        ev, ei = exact_knn(Q, R, k, metric)
        dist, idx = knn_fn(Q, R, k, metric)
        for i in range(n):
            bad += int(list(idx[i]) != ei[i])
            want = [math.sqrt(v) if metric == "l2" else float(v) for v in ev[i]]
            bad += int(list(dist[i]) != want)
    return bad


@pytest.mark.parametrize("mode", ["sort", "select"])
def test_exact_rational(mode):
    assert exact_failures(lambda Q, R, k, mt: oracle.knn(Q, R, k, mt, mode=mode)) == 0


# ---------------------------------------------------------- library reduction
@pytest.mark.parametrize("metric,name", [("l2", "euclidean"), ("l1", "cityblock"), ("linf", "chebyshev")])
def test_scipy_reduction(metric, name):
    from scipy.spatial.distance import cdist

    Q = synthdata.uniform((70, 13), 7, 1)
    R = synthdata.uniform((333, 13), 7, 0)
    k = 25
    D = cdist(Q.astype(np.float64), R.astype(np.float64), name)
    order = np.argsort(D, axis=1, kind="stable")[:, :k]
    dist, idx = oracle.knn(Q, R, k, metric)
    assert np.array_equal(idx, order)
    np.testing.assert_allclose(dist, np.take_along_axis(D, order, 1), rtol=1e-14, atol=0)


# ------------------------------------------------------------------ 1-D case
def two_pointer_1d(q: float, r: np.ndarray, k: int):
    """k nearest in one dimension: expand a window around q over the sorted values."""
    vals, inv = np.unique(r.astype(np.float64), return_inverse=True)
    groups = [[] for _ in vals]
    for j, g in enumerate(inv):
        groups[g].append(j)  # ascending index inside each group
    hi = int(np.searchsorted(vals, q, side="left"))
    lo = hi - 1
    out = []
    while len(out) < k:
        dl = q - vals[lo] if lo >= 0 else math.inf
        dh = vals[hi] - q if hi < len(vals) else math.inf
        if dl < dh:
            take, lo = groups[lo], lo - 1
        elif dh < dl:
            take, hi = groups[hi], hi + 1
        else:  # equal distance on both sides: merge the two groups by index
            take = sorted(groups[lo] + groups[hi])
            lo, hi = lo - 1, hi + 1
        out.extend((min(dl, dh), j) for j in take)
    return [d for d, _ in out[:k]], [j for _, j in out[:k]]


def test_one_dimension_two_pointer():
    Q = synthdata.integer_grid((40, 1), -20, 20, 11, 1) / 2
    R = synthdata.integer_grid((150, 1), -25, 25, 11, 0)
    for metric in METRICS:
        for k in (1, 7, 150):
            dist, idx = oracle.knn(Q, R, k, metric)
            for i in range(Q.shape[0]):
                wd, wi = two_pointer_1d(float(Q[i, 0]), R[:, 0], k)
                assert list(idx[i]) == wi
                assert list(dist[i]) == wd


# ---------------------------------------------------------------- invariants
def test_sort_and_select_modes_identical():
    Q = synthdata.integer_grid((50, 3), 0, 4, 12, 1)
    R = synthdata.integer_grid((300, 3), 0, 4, 12, 0)  # many exact ties
    for metric in METRICS:
        for k in (1, 20, 300):
            a = oracle.knn(Q, R, k, metric, mode="sort")
            b = oracle.knn(Q, R, k, metric, mode="select")
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("metric", METRICS)
def test_invariants(metric):
    Q = synthdata.gmm(40, 9, 4, 0.2, 13, 1)
    R = synthdata.gmm(257, 9, 4, 0.2, 13, 0)
    m = R.shape[0]
    full_d, full_i = oracle.knn(Q, R, m, metric)
    # I1 non-decreasing
    assert np.all(np.diff(full_d, axis=1) >= 0)
    # I3 k = m is a permutation
    assert np.all(np.sort(full_i, axis=1) == np.arange(m))
    # I2 / I5: every k is a prefix of the full order; the k-th distance is the k-th sorted entry
    for k in (1, 2, 20, 100, m):
        d, i = oracle.knn(Q, R, k, metric)
        assert np.array_equal(i, full_i[:, :k]) and np.array_equal(d, full_d[:, :k])
        Dall = oracle.pair_dist(Q, R, np.repeat(np.arange(40), m), np.tile(np.arange(m), 40), metric)
        assert np.array_equal(d[:, -1], np.sort(Dall.reshape(40, m), axis=1)[:, k - 1])
    # I4 k = 1 is the argmin with the lowest index (np.argmin returns the first minimum)
    Dall = oracle.pair_dist(Q, R, np.repeat(np.arange(40), m), np.tile(np.arange(m), 40), metric).reshape(40, m)
    assert np.array_equal(full_i[:, 0], np.argmin(Dall, axis=1))
    # I6 power-of-two scaling: distances scale exactly, indices unchanged
    d2, i2 = oracle.knn(Q * 4, R * 4, 20, metric)
    assert np.array_equal(i2, full_i[:, :20]) and np.array_equal(d2, 4 * full_d[:, :20])
    # I7 permuting R permutes the returned indices (the data has no ties)
    perm = np.random.default_rng(3).permutation(m)
    d3, i3 = oracle.knn(Q, R[perm].copy(), 20, metric)
    assert np.array_equal(perm[i3], full_i[:, :20]) and np.array_equal(d3, full_d[:, :20])
    # I8 translating Q and R together: same neighbours, distances within rounding
    d4, i4 = oracle.knn(Q + 0.5, R + 0.5, 20, metric)
    assert np.array_equal(i4, full_i[:, :20])
    np.testing.assert_allclose(d4, full_d[:, :20], rtol=1e-5)
    # I9 each query's answer does not depend on the other queries
    d5, i5 = oracle.knn(Q[7:9].copy(), R, 20, metric)
    assert np.array_equal(i5, full_i[7:9, :20]) and np.array_equal(d5, full_d[7:9, :20])


def test_metric_inequalities():
    Q = synthdata.uniform((30, 6), 14, 1)
    R = synthdata.uniform((90, 6), 14, 0)
    qi = np.repeat(np.arange(30), 90)
    rj = np.tile(np.arange(90), 30)
    l2 = oracle.pair_dist(Q, R, qi, rj, "l2")
    l1 = oracle.pair_dist(Q, R, qi, rj, "l1")
    li = oracle.pair_dist(Q, R, qi, rj, "linf")
    eps = 1e-12
    assert np.all(li <= l2 + eps) and np.all(l2 <= l1 + eps) and np.all(l1 <= 6 * li + eps)
    assert np.all(l2 <= math.sqrt(6) * li + eps)
    # d = 1: the three metrics coincide
    Q1, R1 = Q[:, :1].copy(), R[:, :1].copy()
    a = [oracle.knn(Q1, R1, 10, mt) for mt in METRICS]
    assert all(np.array_equal(a[0][0], x[0]) and np.array_equal(a[0][1], x[1]) for x in a)


def test_float32_difference_form_within_bound():
    """Closed-form bound: the float32 difference form is within (d/2+2)u (L2), d u (L1), u (Linf).

    This pins the tolerance 1e-5 as attainable for d <= 128 and pins the oracle
    to an independent float32 evaluation of the same definition.
    """
    u = 2.0 ** -24
    for d in (1, 7, 32, 128):
        Q = synthdata.gmm(16, d, 8, 0.05, 15 + d, 1)
        R = synthdata.gmm(200, d, 8, 0.05, 15 + d, 0)
        qi = np.repeat(np.arange(16), 200)
        rj = np.tile(np.arange(200), 16)
        diff = Q[qi] - R[rj]  # float32, exact rounding of each difference
        acc2 = np.zeros(qi.size, np.float32)
        acc1 = np.zeros(qi.size, np.float32)
        accm = np.zeros(qi.size, np.float32)
        for t in range(d):
            acc2 = acc2 + diff[:, t] * diff[:, t]
            acc1 = acc1 + np.abs(diff[:, t])
            accm = np.maximum(accm, np.abs(diff[:, t]))
        for metric, val, bound in (("l2", np.sqrt(acc2), (d / 2 + 2) * u), ("l1", acc1, d * u + u),
                                   ("linf", accm, u)):
            ref = oracle.pair_dist(Q, R, qi, rj, metric)
            rel = np.abs(val.astype(np.float64) - ref) / ref
            assert rel.max() <= bound, (metric, d, rel.max(), bound)
            assert bound < 1e-5 or d > 128


# ------------------------------------------------------------ planted errors
MUTANTS = {
    "tie_break_reversed": ("return a->j < b->j;", "return a->j > b->j;"),
    "sqrt_dropped": ("return metric == ORACLE_L2 ? sqrt(v) : v;", "return v;"),
    "abs_dropped": ("s += fabs(diff);", "s += diff;"),
    "last_dim_dropped": ("for (int32_t t = 0; t < d; ++t) {", "for (int32_t t = 0; t + 1 < d; ++t) {"),
    "sign_flipped": ("double diff = (double)q[t] - (double)r[t];", "double diff = (double)q[t] + (double)r[t];"),
    "heap_keeps_largest": ("} else if (pair_less(&p, &buf[0])) {", "} else if (pair_less(&buf[0], &p)) {"),
    "max_as_sum": ("if (a > s) s = a;", "s += a;"),
    "operands_swapped": ("const float* q = Q + i * (int64_t)d;", "const float* q = R + (i % m) * (int64_t)d;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    """A copy of the oracle with one planted mistake must fail at least one pin."""
    import ctypes

    src = open(os.path.join(os.path.dirname(oracle.__file__), "knn_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1
    so = str(tmp_path / "mutant.so")
    cfile = tmp_path / "mutant.c"
    cfile.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", so, str(cfile), "-lm"])
    lib = ctypes.CDLL(so)
    lib.knn_oracle.argtypes = oracle._load().knn_oracle.argtypes

    def mutant_knn(Q, R, k, metric, mode="select"):
        Q = np.ascontiguousarray(Q, np.float32)
        R = np.ascontiguousarray(R, np.float32)
        n, d = Q.shape
        dist = np.empty((n, k)); idx = np.empty((n, k), np.int64)
        lib.knn_oracle(Q.ctypes.data, n, R.ctypes.data, R.shape[0], d, k, oracle.METRICS[metric],
                       {"sort": 0, "select": 1}[mode], 0, dist.ctypes.data, idx.ctypes.data)
        return dist, idx

    caught = hand_2d_failures(mutant_knn) + exact_failures(mutant_knn, trials=30)
    assert caught > 0, f"planted mistake {name} went unnoticed"
