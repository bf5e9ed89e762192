"""FP64 k-nearest-neighbour entropy estimator (Kozachenko-Leonenko / Goria et
al.), the entropy-estimation application of the paper's Section 2.2.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the GPU library never
imports it.

For points y_1..y_n in R^d, rho_k(y_i) is the distance from y_i to its k-th
nearest neighbour among the other n - 1 points, and

    H_{n,k} = (1/n) sum_i [ d log rho_k(y_i) + log(n - 1) ] + log c_1(d) - Psi(k)

with c_1(d) = 2 pi^(d/2) / (d Gamma(d/2)) the volume of the unit ball (Eq. (5))
and Psi the digamma function (Eq. (4)), Psi(k) = -gamma + sum_{j<k} 1/j for an
integer k.  Reading of Eq. (3): it prints log((n - 1) rho_k(y_i)) with no
power d; the estimator of Goria et al. that the paper cites uses
rho_k(y_i)^d (without it, scaling the data by a shifts the estimate by log a
instead of the d log a of a d-dimensional density), so the term read here is
log((n - 1) rho_k(y_i)^d).
"""
from __future__ import annotations

import math

import numpy as np

from . import knn

EULER_GAMMA = 0.57721566490153286060651209008240243


def digamma_int(k: int) -> float:
    """Psi(k) for a positive integer k: -gamma + sum_{j=1}^{k-1} 1/j."""
    if k < 1:
        raise ValueError("k >= 1")
    return -EULER_GAMMA + math.fsum(1.0 / j for j in range(1, k))


def unit_ball_volume(d: int) -> float:
    """c_1(d) = 2 pi^(d/2) / (d Gamma(d/2)), Eq. (5)."""
    return math.exp(math.log(2.0) + 0.5 * d * math.log(math.pi) - math.log(d) - math.lgamma(0.5 * d))


def kth_neighbour_distance(Y, k: int, threads: int = 0) -> np.ndarray:
    """rho_k(y_i) for every i: the k-th smallest Euclidean distance from y_i to
    the other points (float64).  The brute force returns the k + 1 nearest in
    (distance, index) order, which include y_i itself at distance 0 unless k + 1
    other points coincide with it; removing that one entry leaves the k
    nearest others."""
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    n = Y.shape[0]
    if not 1 <= k <= n - 1:
        raise ValueError("1 <= k <= n - 1")
    dist, idx = knn(Y, Y, k + 1, "l2", threads=threads)
    self_at = idx == np.arange(n)[:, None]
    has_self = self_at.any(axis=1)
    # k-th other neighbour: position k if the point itself is among the first
    # k + 1 (it is then at a position <= k), else position k - 1
    return np.where(has_self, dist[:, k], dist[:, k - 1])


def entropy_knn(Y, k: int, threads: int = 0) -> float:
    """The k-NN entropy estimate H_{n,k}(Y) in nats (Eq. (3), read with rho^d)."""
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    n, d = Y.shape
    rho = kth_neighbour_distance(Y, k, threads)
    with np.errstate(divide="ignore"):
        logs = np.log(rho)
    return float(d * math.fsum(logs) / n + math.log(n - 1) + math.log(unit_ball_volume(d)) - digamma_int(k))
