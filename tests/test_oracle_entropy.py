"""Pins for the FP64 k-NN entropy oracle (``oracle/entropy.py``): checks that
do not trust its own code.  Hand-worked k-th neighbour distances on the line
(self-exclusion, duplicates), the digamma function against scipy, the
unit-ball volume against its closed forms, the estimator against the closed
entropies of the uniform and Gaussian densities (within the statistical error
of the seeded samples), and the exact scaling law H(aY) = H(Y) + d log a that
fixes the power d read into Eq. (3).  The last test plants mistakes in copies
of the estimator and checks that the pins catch each one."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import synthdata
from oracle import entropy as E

HERE = os.path.dirname(os.path.abspath(__file__))


def _cases():
    with open(os.path.join(HERE, "golden", "entropy_line.json")) as f:
        return json.load(f)["cases"]


def rho_failures(fn):
    bad = 0
    for c in _cases():
        Y = np.array(c["points"], dtype=np.float32)[:, None]
        bad += not np.array_equal(fn(Y, c["k"]), np.array(c["rho"], dtype=np.float64))
    return bad


def test_hand_worked_kth_distances():
    assert rho_failures(E.kth_neighbour_distance) == 0


def test_digamma_against_scipy():
    from scipy.special import digamma

    for k in range(1, 60):
        assert abs(E.digamma_int(k) - float(digamma(k))) < 1e-13


def test_unit_ball_volume_closed_forms():
    assert abs(E.unit_ball_volume(1) - 2.0) < 1e-14
    assert abs(E.unit_ball_volume(2) - math.pi) < 1e-14
    assert abs(E.unit_ball_volume(3) - 4.0 * math.pi / 3.0) < 1e-14
    for d in range(3, 40):  # V(d) = 2 pi / d V(d - 2)
        assert abs(E.unit_ball_volume(d) / (2 * math.pi / d * E.unit_ball_volume(d - 2)) - 1) < 1e-12


def uniform_points(n, d, seed):
    return synthdata.uniform((n, d), seed, 0)


def gaussian_points(n, d, sigma, seed):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 5])))
    return (sigma * rng.standard_normal((n, d))).astype(np.float32)


def closed_form_errors(est):
    """Estimator minus the closed-form entropy on seeded samples."""
    errs = []
    # (k >= 2 on the line: 20000 float32 draws from [0, 1) hold a few exact
    # duplicates, whose rho_1 = 0 sends the estimate to -inf)
    for d, k in ((1, 2), (1, 3), (2, 4)):  # uniform on the unit cube: entropy 0
        errs.append(est(uniform_points(20000, d, 60 + d + k), k) - 0.0)
    for d, sigma, k in ((3, 0.5, 4), (4, 1.0, 3)):  # N(0, sigma^2 I): (d/2) log(2 pi e sigma^2)
        errs.append(est(gaussian_points(20000, d, sigma, 70 + d), k) - 0.5 * d * math.log(2 * math.pi * math.e * sigma ** 2))
    return errs


def test_closed_form_entropies():
    """Within the estimator's finite-sample bias and sampling error at
    n = 20000 (a few hundredths of a nat here, growing with d)."""
    errs = closed_form_errors(E.entropy_knn)
    assert max(abs(e) for e in errs) < 0.04, errs


def scaling_errors(est):
    Y = gaussian_points(3000, 4, 1.0, 3)
    h1, h2 = est(Y, 5), est(4.0 * Y, 5)  # exact scaling: 4 is a power of two
    return abs((h2 - h1) - 4 * math.log(4.0))


def test_exact_scaling_law():
    assert scaling_errors(E.entropy_knn) < 1e-9


# ---------------------------------------------------------- planted mistakes
def _no_power_d(Y, k):  # Eq. (3) as printed: log((n-1) rho) without rho^d
    n, d = Y.shape
    rho = E.kth_neighbour_distance(Y, k)
    return float(np.mean(np.log(rho)) + math.log(n - 1) + math.log(E.unit_ball_volume(d)) - E.digamma_int(k))


def _digamma_sign(Y, k):
    n, d = Y.shape
    rho = E.kth_neighbour_distance(Y, k)
    return float(d * np.mean(np.log(rho)) + math.log(n - 1) + math.log(E.unit_ball_volume(d)) + E.digamma_int(k))


def _self_included(Y, k):  # rho taken from the k nearest including the point itself
    from oracle import knn

    dist, _ = knn(np.ascontiguousarray(Y, dtype=np.float32), np.ascontiguousarray(Y, dtype=np.float32), k, "l2")
    return dist[:, k - 1]


def _n_not_n_minus_1(Y, k):
    n, d = Y.shape
    rho = E.kth_neighbour_distance(Y, k)
    return float(d * np.mean(np.log(rho)) + math.log(n) + math.log(E.unit_ball_volume(d)) - E.digamma_int(k))


def test_pins_catch_planted_mistakes():
    assert scaling_errors(_no_power_d) > 1e-3
    assert max(abs(e) for e in closed_form_errors(_digamma_sign)) > 0.5
    assert rho_failures(_self_included) > 0
    # log n instead of log(n - 1) moves the estimate by about 1/n: caught only
    # by an exact reference, here the estimate recomputed term by term on the
    # hand-worked line (k = 1: rho = 1, 1, 2, 4)
    Y = np.array([[0.0], [1.0], [3.0], [7.0]], dtype=np.float32)
    exact = (math.log(1) + math.log(1) + math.log(2) + math.log(4)) / 4 + math.log(3) + math.log(2) + E.EULER_GAMMA
    assert abs(E.entropy_knn(Y, 1) - exact) < 1e-12
    assert abs(_n_not_n_minus_1(Y, 1) - exact) > 1e-3
