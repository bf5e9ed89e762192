"""GPU tests of the batched form: many independent instances in a few launches.

Each instance's result must equal the single-instance search bit for bit (the
scores of a pair do not depend on the launch, and the kept candidates are the
top k' under a total order whatever the slicing), and must pass the
tie-aware oracle check.  Graph replays are compared with the eager result
after eager work of their own in between.
"""
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


def make_instances(seed, count, metrics, storage, dims=(16, 24, 32, 64, 96, 128), ks=(1, 8, 20, 32)):
    import torch

    import paper_0804_1448_amd as K

    rng = np.random.default_rng(seed)
    inst = []
    for i in range(count):
        d = int(rng.choice(dims))
        m = int(rng.integers(100, 6000))
        n = int(rng.integers(1, 700))
        k = int(min(m, rng.choice(ks)))
        metric = metrics[i % len(metrics)]
        R = synthdata.uniform((m, d), 5000 + seed * 1000 + i, 0)
        Q = synthdata.uniform((n, d), 5000 + seed * 1000 + i, 1)
        refs = K.Refs(torch.from_numpy(R).cuda(), storage=storage)
        inst.append(dict(R=R, Q=Q, Qd=torch.from_numpy(Q).cuda(), refs=refs, k=k, metric=metric))
    return inst


def single(inst, precision):
    import torch

    out = []
    for it in inst:
        dist, idx = it["refs"].search(it["Qd"], it["k"], it["metric"], precision=precision)
        out.append((dist, idx))
    torch.cuda.synchronize()
    return [(d.cpu().numpy(), i.cpu().numpy()) for d, i in out]


def as_np(results):
    import torch

    torch.cuda.synchronize()
    return [(d.cpu().numpy(), i.cpu().numpy()) for d, i in results]


@pytest.mark.parametrize("precision,metrics", [("fp32", ["l2", "l1", "linf"]), ("fp16", ["l2"]), ("bf16", ["l2"])])
def test_batched_equals_single_and_oracle(K, precision, metrics):
    banner(f"batched {precision}")
    inst = make_instances(1, 24, metrics, precision)
    want = single(inst, precision)
    got = as_np(K.search_batched([(it["refs"], it["Qd"], it["k"], it["metric"]) for it in inst], precision))
    hits = slots = 0.0
    for j, (it, (wd, wi), (gd, gi)) in enumerate(zip(inst, want, got)):
        assert np.array_equal(wd, gd) and np.array_equal(wi, gi), f"instance {j}"
        rep = compare(it["Q"], it["R"], it["k"], it["metric"], gd, gi, tol=TOL)
        if precision == "fp32":
            assert rep["ok"], (j, rep)
        else:
            # hits within the tolerance, every returned distance that of its index
            assert rep["bad_index_rows"] == 0 and rep["bad_pair"] == 0, (j, rep)
            assert rep["max_rel_err_hits"] <= TOL, (j, rep)
            hits += rep["recall"] * rep["queries"] * rep["k"]
            slots += rep["queries"] * rep["k"]
    if precision != "fp32":
        assert hits / slots >= 0.999, hits / slots  # recall@k pooled over every instance
    for it in inst:
        it["refs"].close()


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_batched_one_launch_equals_per_group_launches(K, precision):
    """All 16-bit instances with k' <= 128 and d <= 128 run in one launch of
    the 32x32-tile kernel (one workgroup per item, items taken longest first
    through a counter).  Its results must equal, bit for bit, those of
    per-group launches (KNN_BATCH_ONE=-1), of one launch per (padded width,
    list size) class (KNN_BATCH_SPLIT=1) and of single searches, for every
    padded width and for lists of one and two keys per lane."""
    import os

    banner(f"batched one launch {precision}")
    inst = make_instances(5, 20, ["l2"], precision, dims=(16, 32, 48, 64, 100, 128), ks=(1, 8, 32, 60, 100))
    probs = [(it["refs"], it["Qd"], it["k"], it["metric"]) for it in inst]
    want = []
    for it in inst:
        d_, i_ = it["refs"].search(it["Qd"], it["k"], "l2", precision=precision, s_extra=28)
        want.append((d_.cpu().numpy(), i_.cpu().numpy()))
    one = as_np(K.search_batched(probs, precision, s_extra=28))
    os.environ["KNN_BATCH_ONE"] = "-1"
    try:
        per_group = as_np(K.search_batched(probs, precision, s_extra=28))
    finally:
        del os.environ["KNN_BATCH_ONE"]
    os.environ["KNN_BATCH_SPLIT"] = "1"  # one launch per (padded width, list size) class
    try:
        split = as_np(K.search_batched(probs, precision, s_extra=28))
    finally:
        del os.environ["KNN_BATCH_SPLIT"]
    hits = slots = 0.0
    for j, (it, (wd, wi), (od, oi), (gd, gi), (sd, si)) in enumerate(zip(inst, want, one, per_group, split)):
        assert np.array_equal(wd, od) and np.array_equal(wi, oi), f"instance {j}: one launch vs single"
        assert np.array_equal(gd, od) and np.array_equal(gi, oi), f"instance {j}: one launch vs per group"
        assert np.array_equal(sd, od) and np.array_equal(si, oi), f"instance {j}: one launch vs per class"
        rep = compare(it["Q"], it["R"], it["k"], "l2", od, oi, tol=TOL)
        assert rep["bad_index_rows"] == 0 and rep["bad_pair"] == 0 and rep["max_rel_err_hits"] <= TOL, (j, rep)
        hits += rep["recall"] * rep["queries"] * rep["k"]
        slots += rep["queries"] * rep["k"]
    assert hits / slots >= 0.999, hits / slots
    for it in inst:
        it["refs"].close()


def test_batched_large_k_and_ragged(K):
    """k' above 64 takes the rank merge; instances with n = 1, m = k and n not a multiple of 16."""
    import torch

    banner("batched large k")
    inst = make_instances(2, 6, ["l2"], "fp32", dims=(32, 80), ks=(100,))
    R = synthdata.uniform((50, 12), 77, 0)
    Q = synthdata.uniform((1, 12), 77, 1)
    import paper_0804_1448_amd as KK

    inst.append(dict(R=R, Q=Q, Qd=torch.from_numpy(Q).cuda(), refs=KK.Refs(torch.from_numpy(R).cuda()), k=50,
                     metric="l2"))
    want = single(inst, "fp32")
    got = as_np(K.search_batched([(it["refs"], it["Qd"], it["k"], it["metric"]) for it in inst], "fp32"))
    for j, (it, (wd, wi), (gd, gi)) in enumerate(zip(inst, want, got)):
        assert np.array_equal(wd, gd) and np.array_equal(wi, gi), f"instance {j}"
        assert compare(it["Q"], it["R"], it["k"], "l2", gd, gi, tol=TOL)["ok"]
    for it in inst:
        it["refs"].close()


def test_batched_graph_replays_match_eager(K):
    import torch

    banner("batched graph")
    inst = make_instances(3, 10, ["l2"], "fp16")
    probs = [(it["refs"], it["Qd"], it["k"], it["metric"]) for it in inst]
    eager = as_np(K.search_batched(probs, "fp16"))
    b = K.Batch(probs, "fp16")
    for rep in range(4):
        b.run(use_graph=True)
        torch.cuda.synchronize()
        got = as_np(b.results())
        for j, ((ed, ei), (gd, gi)) in enumerate(zip(eager, got)):
            assert np.array_equal(ed, gd) and np.array_equal(ei, gi), (rep, j)
        # eager work of the program between replays, and a clobber of the outputs
        for d, i in b.results():
            d.fill_(-1.0)
            i.fill_(-1)
        x = torch.randn(1024, 1024, device="cuda")
        (x @ x).sum().item()
    b.close()
    for it in inst:
        it["refs"].close()


def test_batched_tuning_keeps_results(K):
    banner("batched tuning")
    inst = make_instances(4, 8, ["l2"], "fp16")
    probs = [(it["refs"], it["Qd"], it["k"], it["metric"]) for it in inst]
    plain = as_np(K.search_batched(probs, "fp16"))
    b = K.Batch(probs, "fp16", tune=True)
    b.run()
    tuned = as_np(b.results())
    b.close()
    for (pd, pi), (td, ti) in zip(plain, tuned):
        assert np.array_equal(pd, td) and np.array_equal(pi, ti)
    for it in inst:
        it["refs"].close()
