"""GPU parity of the k-NN entropy estimate (knn_entropy, Section 2.2 Eq. (3)-(5))
against the FP64 oracle (oracle/entropy.py), through the C ABI.

Tolerance: each rho_k is a float32 distance within relative 1e-5 of the
oracle's (the search's own bar), so log rho_k is within about 1e-5 absolute
and the estimate, d times their mean, within d * 1e-5 (plus the double
rounding of the sums).
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import synthdata
from oracle import entropy as E

pytestmark = pytest.mark.gpu


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


def gpu_entropy(K, Y, k):
    import torch

    return K.entropy(torch.from_numpy(np.ascontiguousarray(Y)).cuda(), k)


def gaussian(n, d, sigma, seed):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 9])))
    return (sigma * rng.standard_normal((n, d))).astype(np.float32)


CASES = [
    # (name, n, d, k)
    ("uniform", 4000, 2, 4), ("uniform", 3001, 1, 2), ("gauss", 5000, 3, 1), ("gauss", 5000, 3, 8),
    ("gmm", 3000, 16, 5), ("gmm", 2048, 96, 20), ("gauss", 2, 4, 1), ("gmm", 700, 130, 3),
]


@pytest.mark.parametrize("name,n,d,k", CASES)
def test_entropy_matches_oracle(K, name, n, d, k):
    banner(f"entropy {name} n={n} d={d} k={k}")
    if name == "uniform":
        Y = synthdata.uniform((n, d), 900 + d, 0)
    elif name == "gauss":
        Y = gaussian(n, d, 0.7, 910 + d)
    else:
        Y = synthdata.gmm(n, d, 16, 0.05, 920 + d, 0)
    h_gpu = gpu_entropy(K, Y, k)
    h_ref = E.entropy_knn(Y, k)
    assert abs(h_gpu - h_ref) <= d * 1e-5 + 1e-9 * abs(h_ref), (h_gpu, h_ref)


def test_entropy_duplicates_give_minus_infinity(K):
    """Two coincident points have rho_1 = 0: the estimate is -inf on both sides."""
    Y = synthdata.uniform((500, 3), 930, 0)
    Y[10] = Y[20]
    assert gpu_entropy(K, Y, 1) == -math.inf and E.entropy_knn(Y, 1) == -math.inf
    # with k = 2 the duplicate pair has a positive rho_2 again
    assert abs(gpu_entropy(K, Y, 2) - E.entropy_knn(Y, 2)) <= 3e-5


def test_entropy_rejects_bad_arguments(K):
    import torch

    Y = torch.zeros((5, 3), dtype=torch.float32, device="cuda")
    for k in (0, 5):
        with pytest.raises(K.KnnError):
            K.entropy(Y, k)
    with pytest.raises(K.KnnError):
        K.entropy(Y[:1], 1)
