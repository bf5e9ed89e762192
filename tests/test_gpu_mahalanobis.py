"""GPU parity of the Mahalanobis brute force (knn_search_mahalanobis) against
the FP64 oracle (oracle/mahalanobis.py), through the C ABI.

Check, per query: the returned indices are distinct, and the FP64 Mahalanobis
distance of the neighbour returned at each position, as well as the returned
distance itself, is within relative 1e-5 of the oracle's distance at that
position (so an index may differ from the oracle's only where another
reference lies within the tolerance at that rank).  Sigma = I must give the
Euclidean search's results exactly.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import synthdata
from oracle.mahalanobis import knn_mahalanobis

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


def factor(d, seed, kind):
    """L with Sigma^-1 = L L^T."""
    if kind == "identity":
        return np.eye(d)
    rng = np.random.default_rng(seed)
    if kind == "diagonal":
        return np.diag(rng.uniform(0.5, 2.0, d))
    A = rng.standard_normal((d, d))
    S = A @ A.T / d + np.eye(d)  # a well-conditioned covariance
    return np.linalg.cholesky(np.linalg.inv(S))


def run(K, Q, R, L, k):
    import torch

    c = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    dist, idx = K.search_mahalanobis(c(Q), c(R), c(L), k)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), idx.cpu().numpy()


def check(Q, R, L, k, dist, idx):
    L32 = np.asarray(L, dtype=np.float32).astype(np.float64)  # the float32 factor the GPU used
    D, _ = knn_mahalanobis(Q, R, L32, k)
    assert np.all(np.sort(idx, axis=1)[:, 1:] != np.sort(idx, axis=1)[:, :-1])
    for i in range(Q.shape[0]):
        t = (Q[i].astype(np.float64) - R[idx[i]].astype(np.float64)) @ L32
        true = np.sqrt(np.einsum("ij,ij->i", t, t))
        scale = np.maximum(D[i], 1e-30)
        assert np.all(np.abs(true - D[i]) <= TOL * scale), (i, true, D[i])
        assert np.all(np.abs(dist[i] - D[i]) <= TOL * scale), (i, dist[i], D[i])


CASES = [(64, 2000, 8, 10, "general"), (100, 3000, 16, 20, "diagonal"), (33, 777, 3, 5, "general"),
         (257, 4100, 32, 8, "general"), (10, 500, 96, 12, "general"), (1, 1, 1, 1, "diagonal")]


@pytest.mark.parametrize("n,m,d,k,kind", CASES)
def test_mahalanobis_matches_oracle(K, n, m, d, k, kind):
    banner(f"mahalanobis n={n} m={m} d={d} k={k} {kind}")
    Q, R = synthdata.uniform((n, d), 950 + d, 1), synthdata.uniform((m, d), 950 + d, 0)
    L = factor(d, 960 + d, kind)
    check(Q, R, L, k, *run(K, Q, R, L, k))


def test_identity_equals_euclidean(K):
    """Sigma = I: the Mahalanobis search returns the Euclidean search's
    neighbours (exactly where the oracle separates consecutive neighbours by
    more than 1e-6) and distances within 1e-6."""
    import torch

    import oracle

    banner("mahalanobis identity")
    Q, R = synthdata.uniform((200, 24), 970, 1), synthdata.uniform((3000, 24), 970, 0)
    a = run(K, Q, R, np.eye(24), 15)
    b = [t.cpu().numpy() for t in K.search(torch.from_numpy(Q).cuda(), torch.from_numpy(R).cuda(), 15, "l2")]
    D, _ = oracle.knn(Q, R, 16, "l2")
    separated = np.all(np.diff(D, axis=1) > 1e-6 * D[:, 1:], axis=1)
    assert separated.mean() > 0.9
    assert np.array_equal(a[1][separated], b[1][separated])
    assert np.allclose(a[0], b[0], rtol=1e-6, atol=0)


def test_clustered_data(K):
    """Tight clusters (sigma = 0.01) far from the set's centre: neighbours
    are 30x closer to each other than to the centre, which the exact re-rank
    from the caller's rows must not feel."""
    banner("mahalanobis clustered")
    d = 32
    Q = synthdata.gmm(200, d, 64, 0.01, 980, 1)
    R = synthdata.gmm(20000, d, 64, 0.01, 980, 0)
    L = factor(d, 981, "general")
    check(Q, R, L, 10, *run(K, Q, R, L, 10))


def test_near_duplicates(K):
    """Queries 1e-5 from a reference and references 1e-6 from one another:
    distances of order 1e-5 next to coordinates of order 1 must still come
    out within relative 1e-5."""
    banner("mahalanobis near duplicates")
    d = 24
    R = synthdata.gmm(5000, d, 16, 0.05, 985, 0)
    rng = synthdata.rng_for(985, synthdata.ROLE_EXTRA)
    dup = rng.choice(5000, 500, replace=False)
    R[dup[:250]] = R[dup[250:]] + (1e-6 * rng.standard_normal((250, d))).astype(np.float32)
    Q = (R[dup[250:350]] + 1e-5 * rng.standard_normal((100, d))).astype(np.float32)
    L = factor(d, 986, "general")
    dist, idx = run(K, Q, R, L, 8)
    assert np.all(dist[:, 0] < 1e-3)
    check(Q, R, L, 8, dist, idx)
