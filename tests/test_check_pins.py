"""Pins for the tie-aware checker ``oracle.check.compare``.

Every GPU parity verdict rests on ``compare``: it formalises "the k nearest
references under a given distance" of Section 2.1 as the rules T1 (distances
within the relative tolerance at every rank), T2 (distinct, in-range indices
whose oracle distance matches the oracle's distance at that rank, so only
near-tie groups may be permuted or swapped across the k boundary) and the
pairing rule (a returned distance is the distance to the returned index).

These tests fix it without trusting its code: the oracle's own result and a
permutation inside an exact-tie group must pass; planted mistakes of the kinds
a GPU kernel could make must each fail; recall figures are checked on planted
cases whose value is known by construction; the Wilson interval is checked
against scipy's.  The last test plants mistakes in copies of ``check.py`` and
requires every copy to fail one of the pins above.
"""
from __future__ import annotations

import types

import numpy as np
import pytest

import oracle
import synthdata
from oracle import check as CHECK

TOL = 1e-5
METRICS = ["l2", "l1", "linf"]


def grid_case(seed=3, n=24, m=300, d=3, lo=0, hi=6):
    """Integer-grid points: many exact ties in every metric."""
    rng = synthdata.rng_for(9100 + seed, synthdata.ROLE_EXTRA)
    Q = rng.integers(lo, hi, (n, d)).astype(np.float32)
    R = rng.integers(lo, hi, (m, d)).astype(np.float32)
    return Q, R


def gmm_case(seed=4, n=40, m=2000, d=16):
    Q = synthdata.gmm(n, d, 8, 0.05, 9200 + seed, synthdata.ROLE_QUERIES)
    R = synthdata.gmm(m, d, 8, 0.05, 9200 + seed, synthdata.ROLE_REFS)
    return Q, R


def line_case(second=1.5e-5):
    """d = 1 (the three distances coincide): the query at 0, references at 1,
    1 + ``second`` and then well apart, so that a returned index or distance
    can sit just inside or just outside the tolerance at a rank."""
    Q = np.zeros((1, 1), np.float32)
    R = np.array([[1.0], [1.0 + second]] + [[2.0 + j] for j in range(20)], np.float32)
    return Q, R


def oracle_result(Q, R, k, metric):
    D, I = oracle.knn(Q, R, k, metric)
    return D.astype(np.float32), I.astype(np.int32), (D, I)


def find_gap(D, rel):
    """(row, rank) of a strict gap D[r+1] > D[r] * (1 + rel) with D[r] > 0."""
    for i in range(D.shape[0]):
        for r in range(D.shape[1] - 1):
            if D[i, r] > 0 and D[i, r + 1] > D[i, r] * (1 + rel):
                return i, r
    raise AssertionError("no gap found")


def run(compare, Q, R, k, metric, dist, idx, ref=None, rows=None):
    return compare(Q, R, k, metric, dist, idx, tol=TOL, ref=ref, rows=rows)


# ------------------------------------------------------------ must pass
def accept_oracle_result(compare):
    bad = 0
    for metric in METRICS:
        for Q, R in (gmm_case(), grid_case()):
            dist, idx, ref = oracle_result(Q, R, 10, metric)
            rep = run(compare, Q, R, 10, metric, dist, idx)
            rep2 = run(compare, Q, R, 10, metric, dist, idx, ref=ref)
            sub = np.array([1, 5, 9])
            rep3 = run(compare, Q, R, 10, metric, dist, idx, ref=(ref[0][sub], ref[1][sub]), rows=sub)
            bad += int(not (rep["ok"] and rep2["ok"] and rep3["ok"] and rep["recall"] == 1.0))
    return bad


def accept_tie_permutation(compare):
    """Swap two entries of an exact-tie group inside the top k, and swap an
    index at rank k-1 with a reference tied with it outside the top k."""
    bad = 0
    for metric in METRICS:
        Q, R = grid_case()
        k = 12
        D, I = oracle.knn(Q, R, k + 20, metric)
        dist = D[:, :k].astype(np.float32).copy()
        idx = I[:, :k].astype(np.int32).copy()
        swaps_in = swaps_across = 0
        for i in range(Q.shape[0]):
            for r in range(k - 1):
                if D[i, r] == D[i, r + 1]:
                    idx[i, r], idx[i, r + 1] = idx[i, r + 1], idx[i, r]
                    swaps_in += 1
                    break
            # a reference outside the top k at exactly the k-th distance
            outside = [j for j in range(k, k + 20) if D[i, j] == D[i, k - 1]]
            if outside and idx[i, k - 1] == I[i, k - 1]:
                idx[i, k - 1] = I[i, outside[0]]
                swaps_across += 1
        assert swaps_in > 0 and swaps_across > 0, "the grid case must hold exact ties"
        rep = run(compare, Q, R, k, metric, dist, idx)
        bad += int(not rep["ok"])
        # strict recall counts the substituted references as misses, tie-aware recall as hits
        want = 1.0 - swaps_across / (Q.shape[0] * k)
        bad += int(abs(rep["recall"] - want) > 1e-12) + int(rep["recall_tie"] != 1.0)
    return bad


# ------------------------------------------------------------ must fail
def plant(fn):
    """Plant one mistake in the oracle's own result; return how many
    (metric, case) combinations the checker failed to reject."""
    missed = 0
    for metric in METRICS:
        Q, R = getattr(fn, "case", gmm_case)()
        k = 10
        dist, idx, ref = oracle_result(Q, R, k, metric)
        dist, idx, kwargs = fn(Q, R, k, metric, dist.copy(), idx.copy(), ref)
        rep = run(compare_under_test[0], Q, R, k, metric, dist, idx, **kwargs)
        missed += int(rep["ok"])
    return missed


def m_far_index(Q, R, k, metric, dist, idx, ref):
    # rank 3 of query 5 points at the reference farthest from it (distance kept)
    far = np.argmax(oracle.pair_dist(Q, R, np.full(R.shape[0], 5), np.arange(R.shape[0]), metric))
    idx[5, 3] = far
    return dist, idx, {}


def m_duplicate(Q, R, k, metric, dist, idx, ref):
    idx[7, 4] = idx[7, 3]
    dist[7, 4] = dist[7, 3]
    return dist, idx, {}


def m_duplicate_in_tie(Q, R, k, metric, dist, idx, ref):
    # inside an exact-tie group the repeated index has the right distance at both ranks
    D = ref[0]
    i, r = next((i, r) for i in range(D.shape[0]) for r in range(k - 1) if D[i, r] == D[i, r + 1])
    idx[i, r + 1] = idx[i, r]
    return dist, idx, {}


m_duplicate_in_tie.case = grid_case


def m_near_index(Q, R, k, metric, dist, idx, ref):
    # references 0 and 1 (distances 1 and 1 + 1.5e-5) trade ranks, both
    # returned at 1 + 0.75e-5: T1 and the pairing hold at both ranks, T2 does not
    assert list(idx[0, :2]) == [0, 1]
    idx[0, 0], idx[0, 1] = 1, 0
    dist[0, 0] = dist[0, 1] = np.float32(1.0 + 0.75e-5)
    return dist, idx, {}


m_near_index.case = line_case


def m_pair_split(Q, R, k, metric, dist, idx, ref):
    # references 0 and 1 (0.9e-5 apart) trade indices, and the distance at
    # rank 0 is put 0.9e-5 below the oracle's: T1 and T2 hold at every rank,
    # but the distance at rank 0 is 1.8e-5 away from its index's
    assert list(idx[0, :2]) == [0, 1]
    idx[0, 0], idx[0, 1] = 1, 0
    dist[0, 0] = np.float32(1.0 - 0.9e-5)
    return dist, idx, {}


m_pair_split.case = lambda: line_case(0.9e-5)


def m_out_of_range_high(Q, R, k, metric, dist, idx, ref):
    idx[2, k - 1] = R.shape[0]
    return dist, idx, {}


def m_out_of_range_negative(Q, R, k, metric, dist, idx, ref):
    idx[2, 0] = -1
    return dist, idx, {}


def m_dist_off(Q, R, k, metric, dist, idx, ref):
    dist[11, 6] = np.float32(dist[11, 6] * (1 + 2e-5))
    return dist, idx, {}


def m_dist_nan(Q, R, k, metric, dist, idx, ref):
    dist[1, 1] = np.nan
    return dist, idx, {}


def m_swap_across_k(Q, R, k, metric, dist, idx, ref):
    # the oracle's (k+1)-th reference and distance replace the k-th where the gap exceeds the tolerance
    D, I = oracle.knn(Q, R, k + 1, metric)
    i, _ = find_gap(D[:, k - 1:], 1e-3)
    assert D[i, k] > D[i, k - 1] * (1 + 1e-3)
    idx[i, k - 1] = I[i, k]
    dist[i, k - 1] = np.float32(D[i, k])
    return dist, idx, {}


def m_swap_across_k_dist_kept(Q, R, k, metric, dist, idx, ref):
    D, I = oracle.knn(Q, R, k + 1, metric)
    i, _ = find_gap(D[:, k - 1:], 1e-3)
    idx[i, k - 1] = I[i, k]
    return dist, idx, {}


def m_non_tie_reorder(Q, R, k, metric, dist, idx, ref):
    D = ref[0]
    i, r = find_gap(D, 1e-3)
    dist[i, r], dist[i, r + 1] = dist[i, r + 1], dist[i, r]
    idx[i, r], idx[i, r + 1] = idx[i, r + 1], idx[i, r]
    return dist, idx, {}


def m_pairing(Q, R, k, metric, dist, idx, ref):
    # distances stay the oracle's, but two indices of a non-tied pair trade places
    D = ref[0]
    i, r = find_gap(D, 1e-3)
    idx[i, r], idx[i, r + 1] = idx[i, r + 1], idx[i, r]
    return dist, idx, {}


def m_wrong_row_rows(Q, R, k, metric, dist, idx, ref):
    # results of query 6 stored in row 5, checked through rows=
    dist[5], idx[5] = dist[6], idx[6]
    return dist, idx, {"rows": np.array([1, 5, 9])}


def m_wrong_row_ref(Q, R, k, metric, dist, idx, ref):
    # a precomputed oracle for rows [1, 6, 9] passed for rows [1, 5, 9]
    D, I = oracle.knn(Q[[1, 6, 9]], R, k, metric)
    return dist, idx, {"rows": np.array([1, 5, 9]), "ref": (D, I)}


MISTAKES = {name[2:]: fn for name, fn in globals().items() if name.startswith("m_")}
compare_under_test = [CHECK.compare]


def reject_all(compare):
    compare_under_test[0] = compare
    try:
        return {name: plant(fn) for name, fn in MISTAKES.items()}
    finally:
        compare_under_test[0] = CHECK.compare


def recall_planted(compare):
    """Replace one top-k member per row with a clear non-member: strict and
    tie-aware recall must both be exactly (k - 1) / k, and the check must fail."""
    bad = 0
    Q, R = gmm_case()
    k = 8
    D, I = oracle.knn(Q, R, 200, "l2")
    dist = D[:, :k].astype(np.float32).copy()
    idx = I[:, :k].astype(np.int32).copy()
    idx[:, k - 1] = I[:, 199]
    dist[:, k - 1] = D[:, 199].astype(np.float32)
    assert np.all(D[:, 199] > D[:, k - 1] * (1 + 1e-3))
    rep = run(compare, Q, R, k, "l2", dist, idx)
    bad += int(abs(rep["recall"] - (k - 1) / k) > 1e-12)
    bad += int(abs(rep["recall_tie"] - (k - 1) / k) > 1e-12)
    bad += int(rep["ok"])
    return bad


# ------------------------------------------------------------------ tests
def test_accepts_oracle_result():
    assert accept_oracle_result(CHECK.compare) == 0


def test_accepts_permutation_inside_exact_tie_group():
    assert accept_tie_permutation(CHECK.compare) == 0


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_rejects_planted_mistake(name):
    compare_under_test[0] = CHECK.compare
    assert plant(MISTAKES[name]) == 0, f"compare accepted a result with mistake {name}"


def test_recall_on_planted_misses():
    assert recall_planted(CHECK.compare) == 0


def test_shape_mismatch_raises():
    Q, R = gmm_case()
    dist, idx, _ = oracle_result(Q, R, 5, "l2")
    with pytest.raises(ValueError):
        CHECK.compare(Q, R, 5, "l2", dist[:, :4], idx[:, :4])


@pytest.mark.parametrize("hits,trials", [(0, 10), (5, 10), (997, 1000), (65536, 65536), (65500, 65536)])
def test_wilson_interval_matches_scipy(hits, trials):
    from scipy.stats import binomtest

    lo, hi = CHECK.recall_ci(hits / trials, trials)
    ci = binomtest(hits, trials).proportion_ci(confidence_level=0.95, method="wilson")
    # recall_ci uses z = 1.96; scipy uses the exact 0.975 normal quantile (1.95996...)
    assert abs(lo - ci.low) < 2e-5 and abs(hi - ci.high) < 2e-5, (lo, hi, ci)


# ------------------------------------------------------- planted in the checker
CHECK_MUTANTS = {
    "tolerance_loosened": ("    rep = {\"queries\": int(nq), \"k\": int(k), \"tol\": tol}\n",
                           "    tol = 10 * tol\n    rep = {\"queries\": int(nq), \"k\": int(k), \"tol\": tol}\n"),
    "distinctness_dropped": ("    rep[\"bad_index_rows\"] = int(np.sum(~(np.all(in_range, axis=1) & distinct)))\n",
                             "    rep[\"bad_index_rows\"] = int(np.sum(~np.all(in_range, axis=1)))\n"),
    "t2_on_returned_distance": ("    bad_idx = (np.abs(d64 - Ds) > lim) | ~in_range\n",
                                "    bad_idx = (np.abs(dist - Ds) > lim) | ~in_range\n"),
    "t2_exact_index": ("    bad_idx = (np.abs(d64 - Ds) > lim) | ~in_range\n",
                       "    bad_idx = (idx != Is) | ~in_range\n"),
    "pairing_dropped": ("    bad_pair = ~(np.abs(dist - d64) <= tol * d64) | ~in_range\n",
                        "    bad_pair = ~in_range\n"),
    "nan_passes": [("    bad_dist = ~(np.abs(dist - Ds) <= lim)  # NaN fails\n",
                    "    bad_dist = np.abs(dist - Ds) > lim\n"),
                   ("    bad_pair = ~(np.abs(dist - d64) <= tol * d64) | ~in_range\n",
                    "    bad_pair = (np.abs(dist - d64) > tol * d64) | ~in_range\n")],
    "rows_ignored": ("    dist = dist[rows].astype(np.float64)\n    idx = idx[rows]\n",
                     "    dist = dist[: rows.size].astype(np.float64)\n    idx = idx[: rows.size]\n"),
    "recall_denominator": ("    rep[\"recall\"] = float(hits.sum() / max(1, nq * k))\n",
                           "    rep[\"recall\"] = float(hits.sum() / max(1, nq * (k - 1)))\n"),
    "tie_recall_strict": ("    kth = Ds[:, -1:] * (1 + tol)\n", "    kth = Ds[:, -1:] * (1 - tol)\n"),
}


def load_mutant(name):
    path = CHECK.__file__
    src = open(path).read()
    edits = CHECK_MUTANTS[name]
    for old, new in edits if isinstance(edits, list) else [edits]:
        assert src.count(old) == 1, f"mutant {name}: anchor not found once"
        src = src.replace(old, new)
    mod = types.ModuleType(f"oracle._check_mutant_{name}")
    mod.__package__ = "oracle"
    mod.__file__ = path
    exec(compile(src, f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(CHECK_MUTANTS))
def test_pins_catch_planted_checker_mistake(name):
    mod = load_mutant(name)
    caught = accept_oracle_result(mod.compare) + accept_tie_permutation(mod.compare)
    caught += sum(reject_all(mod.compare).values())
    caught += recall_planted(mod.compare)
    assert caught > 0, f"planted checker mistake {name} went unnoticed"
