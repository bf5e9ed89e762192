"""Pins for the FP64 Mahalanobis oracle (``oracle/mahalanobis.py``): Sigma = I
reduces to the Euclidean oracle (a separate C brute force), a diagonal Sigma
to the Euclidean oracle on coordinates divided by the standard deviations,
and a general Sigma agrees with the quadratic form (q - r)^T Sigma^-1 (q - r)
evaluated with a linear solve against Sigma itself (never forming L).  The
last test plants mistakes (L instead of L^T, squared distances) and checks
that the pins catch them."""
from __future__ import annotations

import numpy as np

import oracle
import synthdata
from oracle.mahalanobis import knn_mahalanobis


def data(n, m, d, seed):
    return synthdata.uniform((n, d), seed, 1), synthdata.uniform((m, d), seed, 0)


def spd(d, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d))
    return A @ A.T + d * np.eye(d)  # a covariance Sigma


def test_identity_is_euclidean():
    Q, R = data(40, 500, 7, 1)
    D, I = knn_mahalanobis(Q, R, np.eye(7), 12)
    D2, I2 = oracle.knn(Q, R, 12, "l2")
    assert np.array_equal(I, I2) and np.allclose(D, D2, rtol=1e-13, atol=0)


def test_diagonal_is_scaled_euclidean():
    Q, R = data(30, 400, 5, 2)
    s = np.array([0.5, 2.0, 4.0, 1.0, 0.25])  # powers of two: the scaled float32 inputs are exact
    L = np.diag(1.0 / s)  # Sigma = diag(s^2), Sigma^-1 = L L^T
    D, I = knn_mahalanobis(Q, R, L, 10)
    D2, I2 = oracle.knn((Q / s).astype(np.float32), (R / s).astype(np.float32), 10, "l2")
    assert np.array_equal(I, I2) and np.allclose(D, D2, rtol=1e-13, atol=0)


def quadratic_form_failures(fn):
    Q, R = data(20, 300, 6, 3)
    S = spd(6, 4)
    L = np.linalg.cholesky(np.linalg.inv(S))  # Sigma^-1 = L L^T
    D, I = fn(Q, R, L, 8)
    bad = 0
    for i in range(Q.shape[0]):
        diff = Q[i].astype(np.float64) - R.astype(np.float64)
        qf = np.einsum("ij,ij->i", diff, np.linalg.solve(S, diff.T).T)  # (q - r)^T Sigma^-1 (q - r)
        order = np.lexsort((np.arange(R.shape[0]), qf))[:8]
        bad += not (np.array_equal(order, I[i]) and np.allclose(D[i], np.sqrt(qf[order]), rtol=1e-10))
    return bad


def test_general_covariance_matches_quadratic_form():
    assert quadratic_form_failures(knn_mahalanobis) == 0


def test_pins_catch_planted_mistakes():
    def transposed(Q, R, L, k):  # ||L (q - r)|| instead of ||L^T (q - r)||
        return knn_mahalanobis(Q, R, np.asarray(L).T, k)

    def squared(Q, R, L, k):  # squared distance returned
        D, I = knn_mahalanobis(Q, R, L, k)
        return D * D, I

    assert quadratic_form_failures(transposed) > 0
    assert quadratic_form_failures(squared) > 0
