"""GPU tests of the serving engine: requests from host memory, batched
continuously onto resident sets, must return exactly what a search of the
request alone returns, and pass the tie-aware oracle check."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import synthdata
from oracle.check import compare

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


def make_sets(K, storage, specs, seed):
    import torch

    out = []
    for i, (m, d) in enumerate(specs):
        R = synthdata.uniform((m, d), 9000 + seed * 10 + i, 0)
        out.append((R, K.Refs(torch.from_numpy(R).cuda(), storage=storage)))
    torch.cuda.synchronize()
    return out


def requests(nsets, d, count, seed, max_n=300, ks=(1, 10, 32)):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        s = int(rng.integers(nsets))
        n = int(rng.integers(1, max_n))
        k = int(rng.choice(ks))
        out.append((s, synthdata.uniform((n, d), 9500 + seed * 100 + i, 1), k))
    return out


def alone(refs, Q, k, precision):
    import torch

    dist, idx = refs.search(torch.from_numpy(Q).cuda(), k, "l2", precision=precision)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), idx.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_server_matches_alone_and_oracle(K, precision):
    banner(f"server {precision}")
    d = 48
    sets = make_sets(K, precision, [(5000, d), (3100, d)], 1)
    reqs = requests(len(sets), d, 40, 2)
    with K.Server([r for _, r in sets], mem_budget=256 << 20, max_batches=3, max_batch_queries=1024,
                  precision=precision) as srv:
        tickets = [srv.submit(s, Q, k) for s, Q, k in reqs]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["batches"] <= len(reqs)
    hits = slots = 0.0
    for j, ((s, Q, k), (gd, gi, lat)) in enumerate(zip(reqs, got)):
        wd, wi = alone(sets[s][1], Q, k, precision)
        assert np.array_equal(wd, gd) and np.array_equal(wi, gi), f"request {j}"
        rep = compare(Q, sets[s][0], k, "l2", gd, gi, tol=TOL)
        if precision == "fp32":
            assert rep["ok"], (j, rep)
        else:
            assert rep["bad_index_rows"] == 0 and rep["bad_pair"] == 0, (j, rep)
            assert rep["max_rel_err_hits"] <= TOL, (j, rep)
            hits += rep["recall"] * rep["queries"] * rep["k"]
            slots += rep["queries"] * rep["k"]
        assert lat > 0
    if precision != "fp32":
        assert hits / slots >= 0.999, hits / slots  # recall@k pooled over every request
    for _, r in sets:
        r.close()


@pytest.mark.parametrize("one_set", [False, True])
def test_server_16bit_sets_mixed_k_match_alone(K, one_set):
    """FP16 sets: requests with k + 32 <= 128 run in multi-set launches (every
    set in one launch; one_set=False), k = 100 (k' = 132) in one-set
    batches; with one_set=True every batch holds one set.  Every request's
    result is bitwise the search of the request alone."""
    banner(f"server fp16 mixed k, one_set={one_set}")
    d = 64
    sets = make_sets(K, "fp16", [(7000, d), (20000, d), (1500, d)], 5)
    reqs = requests(len(sets), d, 36, 6, max_n=400, ks=(1, 20, 96, 100))
    with K.Server([r for _, r in sets], mem_budget=512 << 20, max_batches=2, max_batch_queries=2048,
                  precision="fp16", one_set=one_set) as srv:
        tickets = [srv.submit(s, Q, k) for s, Q, k in reqs]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["batches"] < len(reqs)
    hits = slots = 0.0
    for j, ((s, Q, k), (gd, gi, _)) in enumerate(zip(reqs, got)):
        wd, wi = alone(sets[s][1], Q, k, "fp16")
        assert np.array_equal(wd, gd) and np.array_equal(wi, gi), f"request {j} (set {s}, k {k})"
        rep = compare(Q, sets[s][0], k, "l2", gd, gi, tol=TOL)
        assert rep["bad_index_rows"] == 0 and rep["bad_pair"] == 0 and rep["max_rel_err_hits"] <= TOL, (j, rep)
        hits += rep["recall"] * rep["queries"] * rep["k"]
        slots += rep["queries"] * rep["k"]
    assert hits / slots >= 0.999, hits / slots
    for _, r in sets:
        r.close()


def test_server_tight_budget_serialises(K):
    """A budget that holds one request at a time still answers every request."""
    banner("server tight budget")
    d = 32
    sets = make_sets(K, "fp32", [(4000, d)], 3)
    reqs = requests(1, d, 12, 4, max_n=150, ks=(8,))
    with K.Server([sets[0][1]], mem_budget=1 << 20, max_batches=4, max_batch_queries=256) as srv:
        tickets = [srv.submit(s, Q, k) for s, Q, k in reqs]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["peak_mem_in_flight"] <= 1 << 20
    for (s, Q, k), (gd, gi, _) in zip(reqs, got):
        wd, wi = alone(sets[0][1], Q, k, "fp32")
        assert np.array_equal(wd, gd) and np.array_equal(wi, gi)
    sets[0][1].close()


def test_server_rejects_mismatched_sets(K):
    import torch

    banner("server set checks")
    a = K.Refs(torch.rand(100, 16, device="cuda"), storage="fp32")
    b = K.Refs(torch.rand(100, 24, device="cuda"), storage="fp32")
    c = K.Refs(torch.rand(100, 16, device="cuda"), storage="bf16")
    with pytest.raises(K.KnnError):
        K.Server([a, b], mem_budget=1 << 24)
    with pytest.raises(K.KnnError):
        K.Server([a, c], mem_budget=1 << 24)
    for r in (a, b, c):
        r.close()
