"""GPU parity at the full sizes of the method's larger forms, in the launch
configuration the benchmark times, on sampled query rows that the oracle
computes one by one:

* the precision form: 2^20 references and 65536 queries in 128 dimensions
  from a 1024-cluster Gaussian mixture, k = 32, 16-bit tiles (BF16, FP16)
  with 32 extra candidates and the exact float32 re-rank, and the resident
  float32 search of the same sets (which must pass the strict check);
* the batched form: 512 instances of uneven m, n, d and k, FP16 tiles +
  re-rank, autotuned, replayed from a HIP graph;
* the serving form: four resident FP16 sets of 1-4 Mi points, requests of
  the serving trace batched together, each equal to the request alone.

Bars: no invalid or repeated index; recall@k >= 0.999 for the 16-bit tiles;
distances of the hits within relative 1e-5 of the oracle's; the float32
search passes the tie-aware check outright.
"""
from __future__ import annotations

import os
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


def threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def sample_rows(n, count, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, n - 1], rng.choice(n, size=count, replace=False)]))


@pytest.fixture(scope="module")
def precision_sets():
    import torch

    p = dict(synthdata.WORKLOADS["gmm1m_d128"])
    th = threads()
    R = synthdata.gmm(p["m"], p["d"], p["comps"], p["sigma"], p["wid"], synthdata.ROLE_REFS, threads=th)
    Q = synthdata.gmm(p["n"], p["d"], p["comps"], p["sigma"], p["wid"], synthdata.ROLE_QUERIES, threads=th)
    rows = sample_rows(p["n"], 160, 31)
    import oracle

    ref = oracle.knn(Q[rows], R, p["k"], "l2")
    yield dict(R=R, Q=Q, Rd=torch.from_numpy(R).cuda(), Qd=torch.from_numpy(Q).cuda(), k=p["k"], rows=rows, ref=ref)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_precision_form_full_size(K, precision_sets, prec):
    import torch

    s = precision_sets
    banner(f"precision form {prec}: n={s['Q'].shape[0]} m={s['R'].shape[0]} d=128 k={s['k']} + 32")
    refs = K.Refs(s["Rd"], storage=prec, keep_fp32_master=True)
    try:
        dist, idx = refs.search(s["Qd"], s["k"], "l2", precision=prec, s_extra=32)
        torch.cuda.synchronize()
        dist, idx = dist.cpu().numpy(), idx.cpu().numpy()
    finally:
        refs.close()
    rep = compare(s["Q"], s["R"], s["k"], "l2", dist, idx, tol=TOL, ref=s["ref"], rows=s["rows"])
    assert rep["bad_index_rows"] == 0, rep
    assert rep["recall"] >= 0.999, rep
    assert rep["max_rel_err_hits"] <= TOL and rep["bad_pair"] == 0 and rep["bad_index_rows"] == 0, rep
    assert np.all(np.diff(dist[s["rows"]], axis=1) >= 0)


def test_precision_sets_fp32_full_size(K, precision_sets):
    import torch

    s = precision_sets
    banner("precision sets, resident float32")
    refs = K.Refs(s["Rd"], storage="fp32")
    try:
        dist, idx = refs.search(s["Qd"], s["k"], "l2", precision="fp32")
        torch.cuda.synchronize()
        dist, idx = dist.cpu().numpy(), idx.cpu().numpy()
    finally:
        refs.close()
    rep = compare(s["Q"], s["R"], s["k"], "l2", dist, idx, tol=TOL, ref=s["ref"], rows=s["rows"])
    assert rep["ok"], rep


def test_batched_form_full_size(K):
    import torch
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    specs = synthdata.batch_specs()
    banner(f"batched form: {len(specs)} instances, fp16 + re-rank, tuned, graph replay")
    with ThreadPoolExecutor(threads()) as ex:
        data = list(ex.map(lambda a: synthdata.batch_instance(a[0], *a[1][:3]), enumerate(specs)))
    probs, keep = [], []
    for (m, n, d, k), (R, Q) in zip(specs, data):
        refs = K.Refs(torch.from_numpy(R).cuda(), storage="fp16", keep_fp32_master=True)
        probs.append((refs, torch.from_numpy(Q).cuda(), k, "l2"))
        keep.append(refs)
    # k + 28 <= 128 keeps every instance (k up to 100) in the one launch of
    # the 32x32-tile kernel
    b = K.Batch(probs, "fp16", s_extra=28, tune=True)
    try:
        b.run()
        for _ in range(2):
            b.run(use_graph=True)
        torch.cuda.synchronize()
        outs = b.results()
        rng = np.random.default_rng(17)
        pick = rng.choice(len(specs), size=32, replace=False)
        hits = total = 0
        for i in pick:
            m, n, d, k = specs[i]
            R, Q = data[i]
            rows = sample_rows(n, min(n, 6), 100 + int(i)) if n > 2 else np.arange(n)
            dist, idx = outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy()
            rep = compare(Q, R, k, "l2", dist, idx, tol=TOL, ref=oracle.knn(Q[rows], R, k, "l2"), rows=rows)
            assert rep["bad_index_rows"] == 0, (i, rep)
            assert rep["max_rel_err_hits"] <= TOL and rep["bad_pair"] == 0, (i, rep)
            assert np.all(np.diff(dist[rows], axis=1) >= 0)
            hits += rep["recall"] * len(rows) * k
            total += len(rows) * k
        assert hits / total >= 0.999, hits / total
    finally:
        b.close()
        for r in keep:
            r.close()


def test_serving_form_full_size(K):
    """Four resident FP16 sets of 1-4 Mi points (d = 128); 48 requests of the
    serving trace submitted at once, so that they are batched together and
    their batches overlap on the device.  Each result must equal the same
    request searched alone, bit for bit, and match the oracle on the sets'
    float16-rounded rows (the canonical rows of FP16 storage) on its first
    rows."""
    import torch

    import oracle

    spec = dict(synthdata.SERVE4)
    th = threads()
    extra = 14
    banner(f"serving form: sets {spec['sets']} d={spec['d']}, fp16 + {extra} extra candidates")
    sets, pools = [], []
    for j in range(len(spec["sets"])):
        Rd = torch.from_numpy(synthdata.serve_set(j, spec, threads=th)).cuda()
        sets.append(K.Refs(Rd, storage="fp16", keep_fp32_master=False))
        del Rd
        pools.append(synthdata.serve_queries(j, spec))
    trace = synthdata.serve_requests(48, spec)
    try:
        with K.Server(sets, mem_budget=8 << 30, max_batches=4, max_queue=4096, max_batch_queries=8192,
                      precision="fp16", s_extra=extra) as srv:
            tickets = [srv.submit(s, pools[s][off:off + n], k) for _, s, off, n, k in trace]
            got = [srv.wait(t) for t in tickets]
            st = srv.stats()
        assert st["completed"] == len(trace)
        canon = {}
        recall_num = recall_den = 0.0
        for j, ((_, s, off, n, k), (gd, gi, _)) in enumerate(zip(trace, got)):
            Q = pools[s][off:off + n]
            wd, wi = sets[s].search(torch.from_numpy(Q).cuda(), k, "l2", precision="fp16", s_extra=extra)
            torch.cuda.synchronize()
            assert np.array_equal(wd.cpu().numpy(), gd) and np.array_equal(wi.cpu().numpy(), gi), f"request {j}"
            if j % 4 == 0:
                if s not in canon:
                    canon[s] = synthdata.serve_set(s, spec, threads=th).astype(np.float16).astype(np.float32)
                rows = np.arange(min(n, 8))
                rep = compare(Q, canon[s], k, "l2", gd, gi, tol=TOL,
                              ref=oracle.knn(Q[rows], canon[s], k, "l2", threads=th), rows=rows)
                assert rep["bad_index_rows"] == 0 and rep["bad_pair"] == 0 and rep["max_rel_err_hits"] <= TOL, (j, rep)
                recall_num += rep["recall"] * len(rows)
                recall_den += len(rows)
        assert recall_num / recall_den >= 0.999, recall_num / recall_den
    finally:
        for r in sets:
            r.close()
