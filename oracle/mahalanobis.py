"""FP64 brute-force k-NN under a Mahalanobis distance, one of the distances the
paper's problem definition (Section 2.1) names besides the Euclidean one.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The distance is given by a factor L of the inverse covariance,
Sigma^-1 = L L^T:  d_M(q, r) = sqrt((q - r)^T Sigma^-1 (q - r)) = ||L^T (q - r)||.
Every pair's difference is formed in float64 from the (exactly upcast) float32
inputs, mapped by L^T, and its Euclidean norm taken; the k smallest per query
are kept in (distance, index) order, as in the Euclidean brute force.
"""
from __future__ import annotations

import numpy as np


def knn_mahalanobis(Q, R, L, k: int):
    """Return (dist float64 [n,k], idx int64 [n,k]) for d_M(q, r) = ||L^T (q - r)||."""
    Q = np.asarray(Q, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    n, d = Q.shape
    m = R.shape[0]
    if R.shape[1] != d or L.shape != (d, d) or not 1 <= k <= m:
        raise ValueError("shapes")
    dist = np.empty((n, k))
    idx = np.empty((n, k), dtype=np.int64)
    ref = np.arange(m)
    for i in range(n):
        diff = Q[i][None, :] - R          # q - r for every reference
        t = diff @ L                      # rows (L^T (q - r))^T
        dm = np.sqrt(np.einsum("ij,ij->i", t, t))
        order = np.lexsort((ref, dm))[:k]  # by distance, then index
        dist[i] = dm[order]
        idx[i] = order
    return dist, idx
