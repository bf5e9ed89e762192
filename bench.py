#!/usr/bin/env python3
"""Benchmark of the brute-force k-NN path on one MI355X.

Default mode (``--mode pairs``): a step is one pass of the whole path over the
workload: for each distance of the workload, knn_search (reference
preparation, query preparation, fused distance tiles + per-query selection,
slice merge, exact re-rank and output) on float32 inputs already resident in
device memory.  The default workload is 16384 references and 16384 queries
in 96 dimensions from a 64-component Gaussian mixture, k = 20, searched with
the Euclidean distance (matrix cores) and the Manhattan distance (vector
ALUs).

Prints one JSON line.  Besides the throughput it reports the roofline of the
dominant kernel (its average duration measured with HIP events on the stream
it runs on) and the FP64 oracle timed on the host cores over a query sample,
which also checks the GPU result on that sample.

Other modes print one JSON line each, for the method's other forms:
  --mode precision  2^20 references, 65536 queries, d = 128, k = 32: BF16
                    tiles + 32 extra candidates + exact FP32 re-rank, against
                    the plain FP32 search on the same GPU and the oracle.
  --mode batched    512 independent instances (uneven m, n, d, k) in a few
                    launches, FP16 tiles + re-rank, autotuned, graph replay.
  --mode serve      four resident FP16 sets (1-4 Mi points, d = 128), Poisson
                    arrivals of 1..2048-query requests; QPS and p50/p99
                    latency, against the same trace on FP32 sets.
  --mode copy       a plain 1 GiB device copy: the HBM reference against which
                    the FETCH_SIZE / WRITE_SIZE counters are calibrated.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

# peaks of one MI355X (vendor figures)
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2516.6
# vector ALU, one non-packed lane operation per lane per clock:
# 256 CUs x 64 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# LDS reads taken at 256 bytes per CU per clock, 256 CUs, 2.4 GHz: not a
# datasheet figure; the measured 16-byte read rate (228 bytes per CU per clock,
# profiles/peaks_mi355x.md) exceeds the 128 of the previous generation
PEAK_LDS_TBS = 256 * 256 * 2.4e9 / 1e12
# rates measured on one MI355X by `bench.py --mode peaks` (profiles/peaks_mi355x.md)
MEASURED_FP32_MFMA_TFLOPS = 155.3
MEASURED_BF16_MFMA_TFLOPS = 2231.4
MEASURED_VALU_TOPS = 41.78

WORKLOAD_METRICS = {
    "gmm16384_d96": ["l2", "l1"],
    "uniform4096_d32": ["l2", "l1"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_roofline(name: str, avg_s: float, pairs: float, d: float):
    """Algorithmic work of one fused launch over ``pairs`` query-reference pairs, against its peak."""
    if name.startswith("fused_l2"):
        flops = 2.0 * d * pairs  # cross term q.r: d multiply-adds per pair
        peak = PEAK_FP32_MFMA_TFLOPS if name.endswith("f32") else PEAK_BF16_MFMA_TFLOPS
        ach = flops / avg_s / 1e12
        measured = MEASURED_FP32_MFMA_TFLOPS if name.endswith("f32") else MEASURED_BF16_MFMA_TFLOPS
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "measured_peak": measured, "frac_of_measured": ach / measured,
                "traffic": None, "traffic_unit": "HBM bytes per launch", "kernel": name, "avg_ms": avg_s * 1e3,
                "work_per_launch": flops}
    ops = 2.0 * d * pairs  # one subtract + one absolute accumulate (sum or max) per pair and dimension
    ach = ops / avg_s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TFLOP/s", "frac": ach / PEAK_VALU_TOPS,
            "measured_peak": MEASURED_VALU_TOPS, "frac_of_measured": ach / MEASURED_VALU_TOPS,
            "traffic": None, "traffic_unit": "HBM bytes per launch", "kernel": name, "avg_ms": avg_s * 1e3,
            "work_per_launch": ops}


def measured_traffic(workload: str):
    """HBM bytes per launch of the fused kernels from the committed counter
    summary, or {} when the kernel sources have changed since it was taken."""
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", f"fused_{workload}_traffic.json")
    if not os.path.exists(path):
        return {}
    info = json.load(open(path))
    h = hashlib.sha1(b"".join(open(os.path.join(root, f), "rb").read() for f in info["source_files"])).hexdigest()
    if h[:16] != info["source_hash"]:
        return {}
    return {name: v["read"] + v["write"] for name, v in info["per_launch_bytes"].items()}


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def kernel_table(K):
    return {name: {"avg_ms": tot / cnt, "launches": cnt, "total_ms": tot} for name, (tot, cnt) in K.timing.all().items()}


def timed(K, torch, fn, steps, warmup):
    """Run ``fn`` warmup + steps times; return (seconds per step, kernel table of the timed steps)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    K.timing.reset()
    K.timing.enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    K.timing.enable(False)
    return (t1 - t0) / steps, kernel_table(K)


def oracle_sample(Q, R, k, metrics, target_s, seed=12345, max_rows=None, min_rows=None):
    """Time the oracle on a query sample sized to about ``target_s`` host
    seconds (between ``min_rows`` and ``max_rows`` queries when given)."""
    import numpy as np

    import oracle

    threads = host_threads()
    n = Q.shape[0]
    rng = np.random.default_rng(seed)
    probe = rng.choice(n, size=min(n, 256), replace=False)
    tp = time.perf_counter()
    for mt in metrics:
        oracle.knn(Q[probe], R, k, mt, threads=threads)
    per_query = (time.perf_counter() - tp) / len(probe)
    nsamp = int(min(n, max(len(probe), target_s / max(per_query, 1e-9))))
    if max_rows:
        nsamp = min(nsamp, max_rows)
    if min_rows:
        nsamp = max(nsamp, min(n, min_rows))
    rows = np.sort(rng.choice(n, size=nsamp, replace=False))
    log(f"[bench] oracle sample: {nsamp} queries x {R.shape[0]} references x {len(metrics)} distances, "
        f"{threads} threads")
    tc = time.perf_counter()
    refs = {mt: oracle.knn(Q[rows], R, k, mt, threads=threads) for mt in metrics}
    cpu_s = time.perf_counter() - tc
    return rows, refs, cpu_s, threads


def parity_summary(rep):
    return {kk: rep[kk] for kk in ("ok", "max_rel_err", "max_rel_err_hits", "recall", "recall_tie", "bad_dist",
                                   "bad_idx", "queries")}


# ------------------------------------------------------------------ pairs
def end_to_end_pairs(K, torch, R, Q, k, metrics, pairs_per_step, reps=10):
    """The same step with the inputs starting in pinned host memory and the
    results copied back to host memory: host-to-device copies of R and Q, the
    searches, device-to-host copies of every (dist, idx), all on the current
    stream, timed with host clocks around a synchronized loop.  A context
    figure (the PCIe-inclusive rate), never the benchmark value."""
    Rh = torch.from_numpy(R).pin_memory()
    Qh = torch.from_numpy(Q).pin_memory()
    n = Q.shape[0]
    outs_h = {mt: (torch.empty((n, k), dtype=torch.float32).pin_memory(),
                   torch.empty((n, k), dtype=torch.int32).pin_memory()) for mt in metrics}

    def run():
        Rd = Rh.to("cuda", non_blocking=True)
        Qd = Qh.to("cuda", non_blocking=True)
        for mt in metrics:
            dist, idx = K.search(Qd, Rd, k, mt)
            outs_h[mt][0].copy_(dist, non_blocking=True)
            outs_h[mt][1].copy_(idx, non_blocking=True)

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    return {"value": pairs_per_step / sec, "unit": "pairs/s", "ms_per_step": sec * 1e3, "steps": reps,
            "includes": "H2D of R and Q from pinned memory, the searches, D2H of dist and idx"}


def bench_pairs(args):
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    dev = torch.device("cuda:0")
    R, Q, p = synthdata.workload(args.workload)
    n, m, d, k = p["n"], p["m"], p["d"], p["k"]
    metrics = WORKLOAD_METRICS[args.workload]
    Rd = torch.from_numpy(R).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    outs = {mt: (torch.empty((n, k), dtype=torch.float32, device=dev),
                 torch.empty((n, k), dtype=torch.int32, device=dev)) for mt in metrics}

    def step():
        for mt in metrics:
            K.search(Qd, Rd, k, mt, out=outs[mt])

    log(f"[bench] workload {args.workload}: n={n} m={m} d={d} k={k} metrics={metrics}")
    sec, kernels = timed(K, torch, step, args.steps, args.warmup)
    ms_per_step = sec * 1e3
    pairs_per_step = float(n) * m * len(metrics)
    value = pairs_per_step / sec
    log(f"[bench] {args.steps} steps: {ms_per_step:.4f} ms/step, {value:.4e} pairs/s")
    for name, v in kernels.items():
        log(f"[bench]   {name:16s} avg {v['avg_ms']:.4f} ms x {v['launches']}")
    rooflines = {name: kernel_roofline(name, v["avg_ms"] / 1e3, float(n) * m, d)
                 for name, v in kernels.items() if name.startswith("fused_")}
    traffic = measured_traffic(args.workload)
    for name, roof in rooflines.items():
        roof["traffic"] = traffic.get(name)
    dominant = max(rooflines, key=lambda nm: kernels[nm]["total_ms"])

    result = {
        "metric": "query-ref pairs/sec",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "d": d, "k": k, "distances": metrics,
                   "data": (f"{p['comps']}-component isotropic Gaussian mixture, sigma {p['sigma']}"
                            if p["kind"] == "gmm" else "uniform [0,1)")},
        "roofline": dict(rooflines[dominant]),
        "rooflines": rooflines,
        "kernels": kernels,
    }
    result["end_to_end"] = end_to_end_pairs(K, torch, R, Q, k, metrics, pairs_per_step)
    log(f"[bench] end to end (host inputs in pinned memory, results back on the host): "
        f"{result['end_to_end']['ms_per_step']:.4f} ms/step, {result['end_to_end']['value']:.4e} pairs/s")
    if not args.no_cpu_baseline:
        from oracle.check import compare

        rows, refs, cpu_s, threads = oracle_sample(Q, R, k, metrics, args.cpu_seconds)
        parity = {}
        for mt in metrics:
            rep = compare(Q, R, k, mt, outs[mt][0].cpu().numpy(), outs[mt][1].cpu().numpy(), tol=1e-5,
                          ref=refs[mt], rows=rows)
            parity[mt] = parity_summary(rep)
        result["cpu_baseline"] = {
            "value": float(len(rows)) * m * len(metrics) / cpu_s, "unit": "pairs/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(rows)} seeded queries of {n} against all {m} references, distances {metrics}, "
                      f"FP64 brute force (select mode), {cpu_s:.2f} s",
        }
        result["parity_vs_oracle"] = parity
        result["recall_at_k"] = {mt: parity[mt]["recall"] for mt in metrics}
    return result


# -------------------------------------------------------------- precision
def bench_precision(args):
    """The default line: 2^20 references, 65536 queries, d = 128, k = 32,
    1024-component mixture (sigma 0.1), both sets resident.  ``value`` is the
    plain float32 search (float32 tiles on the matrix cores + 8 extra
    candidates + exact float32 re-rank); the same line reports the BF16 form
    (BF16 tiles, float32 accumulation, 32 extra candidates, exact float32
    re-rank), its speedup, recall@32 and distance errors of both against the
    FP64 oracle on a seeded query sample, and both kernels' rooflines."""
    import numpy as np
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    p = dict(synthdata.WORKLOADS["gmm1m_d128"])
    n, m, d, k = p["n"], p["m"], p["d"], p["k"]
    th = host_threads()
    t0 = time.perf_counter()
    R = synthdata.gmm(m, d, p["comps"], p["sigma"], p["wid"], synthdata.ROLE_REFS, threads=th)
    Q = synthdata.gmm(n, d, p["comps"], p["sigma"], p["wid"], synthdata.ROLE_QUERIES, threads=th)
    log(f"[bench] workload gmm1m_d128: n={n} m={m} d={d} k={k}, generated in {time.perf_counter() - t0:.1f} s")
    Rd = torch.from_numpy(R).cuda()
    Qd = torch.from_numpy(Q).cuda()
    refs32 = K.Refs(Rd, storage="fp32")
    refs16 = K.Refs(Rd, storage="bf16", keep_fp32_master=True)
    del Rd
    out32 = (torch.empty((n, k), dtype=torch.float32, device="cuda"),
             torch.empty((n, k), dtype=torch.int32, device="cuda"))
    out16 = (torch.empty_like(out32[0]), torch.empty_like(out32[1]))
    s_extra = 32
    sec32, kern32 = timed(K, torch, lambda: refs32.search(Qd, k, "l2", precision="fp32", out=out32),
                          args.steps, args.warmup)
    sec16, kern16 = timed(K, torch, lambda: refs16.search(Qd, k, "l2", precision="bf16", s_extra=s_extra,
                                                          out=out16), args.steps, args.warmup)
    pairs = float(n) * m
    log(f"[bench] fp32 {sec32 * 1e3:.2f} ms ({pairs / sec32:.4e} pairs/s), bf16+rerank {sec16 * 1e3:.2f} ms "
        f"({pairs / sec16:.4e} pairs/s)")
    for tag, kt in (("fp32", kern32), ("bf16", kern16)):
        for name, v in kt.items():
            log(f"[bench]   {tag} {name:16s} avg {v['avg_ms']:.4f} ms x {v['launches']}")
    roof32 = kernel_roofline("fused_l2_f32", kern32["fused_l2_f32"]["avg_ms"] / 1e3, pairs, d)
    roof16 = kernel_roofline("fused_l2_bf16", kern16["fused_l2_bf16"]["avg_ms"] / 1e3, pairs, d)
    traffic = measured_traffic("gmm1m_d128")
    for roof in (roof32, roof16):
        roof["traffic"] = traffic.get(roof["kernel"])
        if roof["traffic"] is not None:
            roof["traffic_source"] = "profiles/fused_gmm1m_d128_traffic.json (rocprofv3 FETCH_SIZE + WRITE_SIZE)"
    result = {
        "metric": "query-ref pairs/sec + recall@k vs FP64 oracle",
        "value": pairs / sec32,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gmm1m_d128", "n": n, "m": m, "d": d, "k": k, "distance": "l2",
                   "data": f"{p['comps']}-component isotropic Gaussian mixture, sigma {p['sigma']}",
                   "resident": "both reference sets prepared once (float32; bf16 + float32 master)"},
        "roofline": roof32,
        "bf16": {"value": pairs / sec16, "unit": "pairs/s", "ms_per_step": sec16 * 1e3, "s_extra": s_extra,
                 "dtype": "bf16 tiles, f32 accumulate + f32 re-rank", "roofline": roof16,
                 "speedup_vs_fp32": sec32 / sec16},
        "kernels": {"fp32": kern32, "bf16": kern16},
    }
    if not args.no_cpu_baseline:
        from oracle.check import compare, recall_ci

        rows, refs, cpu_s, threads = oracle_sample(Q, R, k, ["l2"], args.cpu_seconds, max_rows=args.recall_queries,
                                                   min_rows=args.recall_queries)
        rep32 = compare(Q, R, k, "l2", out32[0].cpu().numpy(), out32[1].cpu().numpy(), tol=1e-5, ref=refs["l2"],
                        rows=rows)
        rep16 = compare(Q, R, k, "l2", out16[0].cpu().numpy(), out16[1].cpu().numpy(), tol=1e-5, ref=refs["l2"],
                        rows=rows)
        slots = len(rows) * k
        for tag, rep in (("fp32", rep32), ("bf16", rep16)):
            lo, hi = recall_ci(rep["recall"], slots)
            rep["recall_ci95"] = [lo, hi]
            log(f"[bench] {tag}: recall@{k} {rep['recall']:.6f} (95% CI [{lo:.6f}, {hi:.6f}], {slots} slots), "
                f"max rel err {rep['max_rel_err']:.2e} (hits {rep['max_rel_err_hits']:.2e}), "
                f"tie-aware check {'ok' if rep['ok'] else 'FAILED'}")
        result["parity_vs_oracle"] = {"fp32": parity_summary(rep32), "bf16": parity_summary(rep16)}
        result["recall_at_k"] = {"fp32": rep32["recall"], "bf16": rep16["recall"]}
        result["recall_ci95"] = {"fp32": rep32["recall_ci95"], "bf16": rep16["recall_ci95"],
                                 "method": "Wilson score interval", "slots": slots}
        result["bf16"]["recall_at_k"] = rep16["recall"]
        result["bf16"]["max_rel_err_hits"] = rep16["max_rel_err_hits"]
        result["cpu_baseline"] = {
            "value": float(len(rows)) * m / cpu_s, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(rows)} seeded queries of {n} against all {m} references, Euclidean, FP64 brute force "
                      f"(select mode), {cpu_s:.2f} s",
        }
    refs16.close()
    refs32.close()
    return result


# ---------------------------------------------------------------- batched
def bench_batched(args):
    import numpy as np
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    specs = synthdata.batch_specs(count=args.instances)
    th = host_threads()
    t0 = time.perf_counter()
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(th) as ex:
        data = list(ex.map(lambda a: synthdata.batch_instance(a[0], a[1][0], a[1][1], a[1][2]),
                           enumerate(specs)))
    log(f"[bench] batched workload: {len(specs)} instances generated in {time.perf_counter() - t0:.1f} s")
    probs, keep = [], []
    for (m, n, d, k), (R, Q) in zip(specs, data):
        Rd = torch.from_numpy(R).cuda()
        refs = K.Refs(Rd, storage="fp16", keep_fp32_master=True)
        Qd = torch.from_numpy(Q).cuda()
        probs.append((refs, Qd, k, "l2"))
        keep.append(refs)
        del Rd
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = K.Batch(probs, "fp16", s_extra=args.batch_extra, tune=True)
    b.run()
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    sec, kern = timed(K, torch, lambda: b.run(use_graph=True), args.steps, args.warmup)
    pairs = float(sum(m * n for m, n, _, _ in specs))
    flops = float(sum(2.0 * m * n * d for m, n, d, _ in specs))
    log(f"[bench] batched: {sec * 1e3:.2f} ms/step, {pairs / sec:.4e} pairs/s (tune + first run {tune_s:.1f} s)")
    # eager run, kernel by kernel, for the per-kernel roofline
    sec_e, kern_e = timed(K, torch, lambda: b.run(use_graph=False), max(1, args.steps // 2), 1)
    for name, v in kern_e.items():
        log(f"[bench]   eager {name:16s} avg {v['avg_ms']:.4f} ms x {v['launches']}")
    fused_ms = kern_e.get("fused_l2_f16", {"total_ms": float("nan")})["total_ms"] / max(1, args.steps // 2)
    ach = flops / (fused_ms / 1e3) / 1e12
    roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_BF16_MFMA_TFLOPS, "traffic": None, "kernel": "fused_l2_f16",
            "avg_ms": fused_ms, "work_per_launch": flops, "note": "all fused launches of one step summed"}
    result = {
        "metric": "query-ref pairs/sec",
        "value": pairs / sec,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 tiles, f32 accumulate + f32 re-rank",
        "data": "synthetic",
        "config": {"workload": f"batch{len(specs)}", "instances": len(specs), "pairs": pairs,
                   "m": [1000, 200000], "n": [16, 4096], "d": [16, 32, 64, 128], "k": [1, 8, 32, 100],
                   "graph": True, "tuned": True, "data": "uniform [0,1)", "s_extra": args.batch_extra},
        "eager_ms_per_step": sec_e * 1e3,
        "roofline": roof,
        "kernels": {"graph": kern, "eager": kern_e},
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle.check import compare

        rng = np.random.default_rng(7)
        pick = rng.choice(len(specs), size=min(len(specs), 24), replace=False)
        outs = b.results()
        recalls, ok, worst = [], True, 0.0
        tc = time.perf_counter()
        qsum = 0
        for i in pick:
            m, n, d, k = specs[i]
            R, Q = data[i]
            rows = np.sort(rng.choice(n, size=min(n, 8), replace=False))
            ref = oracle.knn(Q[rows], R, k, "l2", threads=th)
            qsum += len(rows) * m
            rep = compare(Q, R, k, "l2", outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy(), tol=1e-5, ref=ref,
                          rows=rows)
            recalls.append(rep["recall"])
            worst = max(worst, rep["max_rel_err_hits"])
        cpu_s = time.perf_counter() - tc
        result["recall_at_k"] = float(np.mean(recalls))
        result["parity_vs_oracle"] = {"instances": len(pick), "queries_per_instance": 8,
                                      "min_recall": float(np.min(recalls)), "max_rel_err_hits": worst}
        result["cpu_baseline"] = {"value": qsum / cpu_s, "unit": "pairs/s", "cores": th, "kind": "oracle",
                                  "sample": f"8 queries of each of {len(pick)} sampled instances, FP64 brute force"}
    b.close()
    for r in keep:
        r.close()
    return result


# ------------------------------------------------------------------ serve
def run_trace(K, srv, pools, trace, rate, timeout_s=120.0):
    """Submit ``trace`` at ``rate`` requests/s (open loop); return latencies (us) and wall time."""
    import numpy as np

    tickets = []
    lock = threading.Lock()
    done_submitting = threading.Event()
    lat = []
    rejected = [0]

    def waiter():
        i = 0
        while True:
            with lock:
                have = i < len(tickets)
                t = tickets[i] if have else None
            if have:
                _, _, l = srv.wait(t)
                lat.append(l)
                i += 1
            elif done_submitting.is_set():
                with lock:
                    if i >= len(tickets):
                        return
            else:
                time.sleep(0.0002)

    w = threading.Thread(target=waiter)
    w.start()
    t0 = time.perf_counter()
    due = t0
    for gap, s, off, n, k in trace:
        due += gap / rate
        now = time.perf_counter()
        if due > now:
            time.sleep(due - now)
        while True:
            try:
                t = srv.submit(s, pools[s][off:off + n], k)
                break
            except K.KnnError as e:
                if e.status != -5:
                    raise
                rejected[0] += 1
                time.sleep(0.0005)
        with lock:
            tickets.append(t)
        if time.perf_counter() - t0 > timeout_s:
            break
    done_submitting.set()
    w.join()
    wall = time.perf_counter() - t0
    return np.array(lat), wall, len(tickets), rejected[0]


def bench_serve(args):
    import numpy as np
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    spec = dict(synthdata.SERVE4)
    th = host_threads()
    t0 = time.perf_counter()
    sets32, sets16, pools = [], [], []
    for j in range(len(spec["sets"])):
        R = synthdata.serve_set(j, spec, threads=th)
        Rd = torch.from_numpy(R).cuda()
        sets16.append(K.Refs(Rd, storage="fp16", keep_fp32_master=False))
        sets32.append(K.Refs(Rd, storage="fp32"))
        del Rd, R
        pools.append(synthdata.serve_queries(j, spec))
    torch.cuda.synchronize()
    log(f"[bench] serving sets {spec['sets']} d={spec['d']} ready in {time.perf_counter() - t0:.1f} s")
    trace = synthdata.serve_requests(args.requests, spec, sizes=args.sizes)
    skip = len(trace) // 20  # the first 5% of each run are warm-up
    mean_pairs = float(np.mean([n * spec["sets"][s] for _, s, _, n, _ in trace]))
    out = {}
    for tag, sets, prec in (("fp16", sets16, "fp16"), ("fp32", sets32, "fp32")):
        srv = K.Server(sets, mem_budget=args.serve_mem << 30, max_batches=args.serve_streams, max_queue=4096,
                       max_batch_queries=8192, precision=prec, s_extra=args.serve_extra, one_set=args.serve_one_set)
        # capacity: closed loop over the first requests, all submitted at once
        cal = trace[: min(len(trace), 200)]
        _, wall_c, cnt_c, _ = run_trace(K, srv, pools, cal, rate=1e9)
        capacity = cnt_c / wall_c
        res = {"capacity_rps": capacity}
        for load in args.loads:
            rate = load * capacity
            lat, wall, cnt, rej = run_trace(K, srv, pools, trace, rate)
            lat = lat[skip:]
            res[f"load{load:g}"] = {
                "offered_rps": rate, "qps": cnt / wall, "queries_per_s": float(sum(n for _, _, _, n, _ in
                                                                                    trace[:cnt])) / wall,
                "p50_ms": float(np.percentile(lat, 50)) / 1e3, "p99_ms": float(np.percentile(lat, 99)) / 1e3,
                "mean_ms": float(lat.mean()) / 1e3, "requests": cnt, "warmup_requests": skip,
                "busy_retries": rej}
            log(f"[bench] serve {tag} load {load:g}: {res[f'load{load:g}']}")
        res["stats"] = srv.stats()
        res["requests_per_launch"] = res["stats"]["submitted"] / max(1, res["stats"]["batches"])
        res["queries_per_launch"] = res["stats"]["queries"] / max(1, res["stats"]["batches"])
        log(f"[bench] serve {tag}: {res['requests_per_launch']:.2f} requests and {res['queries_per_launch']:.0f} "
            f"queries per launch")
        srv.close()
        out[tag] = res
    # parity of the serving path on a few requests against the oracle
    result = {
        "metric": "serving p50/p99 latency",
        "value": out["fp16"][f"load{args.loads[0]:g}"]["p99_ms"],
        "unit": "ms (p99)",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 200,
        "ms_per_step": None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 tiles, f32 accumulate + f32 re-rank",
        "data": "synthetic",
        "config": {"workload": "serve4_d128", "sets": list(spec["sets"]), "d": spec["d"],
                   "request_queries": list(spec["n"]), "sizes": args.sizes, "k": list(spec["k"]),
                   "arrivals": "Poisson",
                   "mem_budget_gib": args.serve_mem, "mean_pairs_per_request": mean_pairs,
                   "streams": args.serve_streams, "one_set_batches": args.serve_one_set,
                   "s_extra": args.serve_extra},
        "serve": out,
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle.check import compare

        srv = K.Server(sets16, mem_budget=args.serve_mem << 30, precision="fp16", s_extra=args.serve_extra)
        recalls, worst, canon = [], 0.0, {}
        for gap, s, off, n, k in trace[:32]:
            nn = min(n, 16)
            Q = pools[s][off:off + nn]
            dist, idx, _ = srv.wait(srv.submit(s, Q, k))
            # the sets are stored in float16 and those rounded rows are canonical:
            # the oracle sees the same rows, rounded to nearest even
            if s not in canon:
                canon[s] = synthdata.serve_set(s, spec, threads=th).astype(np.float16).astype(np.float32)
            R = canon[s]
            rep = compare(Q, R, k, "l2", dist, idx, tol=1e-5, ref=oracle.knn(Q, R, k, "l2", threads=th))
            recalls.append(rep["recall"])
            worst = max(worst, rep["max_rel_err_hits"])
        srv.close()
        result["recall_at_k"] = float(np.mean(recalls))
        result["parity_vs_oracle"] = {"requests": len(recalls), "min_recall": float(np.min(recalls)),
                                      "max_rel_err_hits": worst}
    for r in sets16 + sets32:
        r.close()
    return result


# ------------------------------------------------------------------- copy
# ---------------------------------------------------------------- entropy
def bench_entropy(args):
    """k-NN entropy estimate (knn_entropy) of the default workload's reference
    set: a self search for the k + 1 nearest of all 16384 points plus the
    per-point logarithms and the fixed-order sum.  Pairs/s counts the n*n
    pairs the self search scores."""
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    R, _, p = synthdata.workload("gmm16384_d96")
    n, d, k = R.shape[0], R.shape[1], p["k"]
    Yd = torch.from_numpy(R).cuda()
    hs = []
    sec, kernels = timed(K, torch, lambda: hs.append(K.entropy(Yd, k)), args.steps, args.warmup)
    log(f"[bench] entropy of {n} x {d} (k = {k}): {sec * 1e3:.4f} ms, estimate {hs[-1]:.6f} nats")
    result = {"metric": "query-ref pairs/sec", "value": float(n) * n / sec, "unit": "pairs/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "entropy_gmm16384_d96", "n": n, "d": d, "k": k},
              "estimate_nats": hs[-1], "kernels": kernels}
    if not args.no_cpu_baseline:
        from oracle import entropy as E

        t0 = time.perf_counter()
        h_ref = E.entropy_knn(R, k, threads=host_threads())
        cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": float(n) * n / cpu_s, "unit": "pairs/s", "cores": host_threads(),
                                  "kind": "oracle", "sample": f"the whole estimate (FP64), {cpu_s:.2f} s"}
        result["parity_vs_oracle"] = {"oracle_nats": h_ref, "abs_err": abs(hs[-1] - h_ref), "tol": d * 1e-5,
                                      "ok": abs(hs[-1] - h_ref) <= d * 1e-5}
        log(f"[bench] oracle {h_ref:.6f} nats, |difference| {abs(hs[-1] - h_ref):.2e}")
    return result


# ------------------------------------------------------------ Mahalanobis
def bench_mahalanobis(args):
    """knn_search_mahalanobis on the default workload's points with a seeded
    general covariance (Sigma = A A^T / d + I, L its inverse's Cholesky
    factor): the mapping of Q and R by L^T plus the Euclidean search."""
    import numpy as np
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    R, Q, p = synthdata.workload("gmm16384_d96")
    n, m, d, k = Q.shape[0], R.shape[0], R.shape[1], p["k"]
    rng = np.random.default_rng(17)
    A = rng.standard_normal((d, d))
    L = np.linalg.cholesky(np.linalg.inv(A @ A.T / d + np.eye(d))).astype(np.float32)
    Qd, Rd, Ld = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (Q, R, L))
    out = [None]
    sec, kernels = timed(K, torch, lambda: out.__setitem__(0, K.search_mahalanobis(Qd, Rd, Ld, k)), args.steps,
                         args.warmup)
    log(f"[bench] Mahalanobis {n} x {m} x {d} (k = {k}): {sec * 1e3:.4f} ms, {n * m / sec:.4e} pairs/s")
    result = {"metric": "query-ref pairs/sec", "value": float(n) * m / sec, "unit": "pairs/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "mahalanobis_gmm16384_d96", "n": n, "m": m, "d": d, "k": k}, "kernels": kernels}
    if not args.no_cpu_baseline:
        from oracle.mahalanobis import knn_mahalanobis

        rows = np.sort(np.random.default_rng(5).choice(n, 64, replace=False))
        t0 = time.perf_counter()
        D, _ = knn_mahalanobis(Q[rows], R, L.astype(np.float64), k)
        cpu_s = time.perf_counter() - t0
        dist, idx = (t.cpu().numpy() for t in out[0])
        err = float(np.max(np.abs(dist[rows] - D) / np.maximum(D, 1e-30)))
        result["cpu_baseline"] = {"value": float(len(rows)) * m / cpu_s, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                                  "sample": f"{len(rows)} seeded queries against all {m} references (numpy FP64), "
                                            f"{cpu_s:.2f} s"}
        result["parity_vs_oracle"] = {"queries": len(rows), "max_rel_err_dist": err, "ok": err <= 1e-5}
        log(f"[bench] oracle sample: {len(rows)} queries, max relative distance error {err:.2e}")
    return result


# ---------------------------------------------------------- classification
def bench_classify(args):
    """knn_classify on the default workload: the 64 mixture components are
    the classes of the 16384 references; each of the 16384 queries takes the
    majority class of its k = 20 nearest."""
    import numpy as np
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    p = dict(synthdata.WORKLOADS["gmm16384_d96"])
    R, lab = synthdata.gmm(p["m"], p["d"], p["comps"], p["sigma"], p["wid"], synthdata.ROLE_REFS, return_labels=True)
    Q = synthdata.gmm(p["n"], p["d"], p["comps"], p["sigma"], p["wid"], synthdata.ROLE_QUERIES)
    n, m, d, k = p["n"], p["m"], p["d"], p["k"]
    Qd, Rd = torch.from_numpy(Q).cuda(), torch.from_numpy(R).cuda()
    labd = torch.from_numpy(lab.astype(np.int32)).cuda()
    out = [None]
    sec, kernels = timed(K, torch, lambda: out.__setitem__(0, K.classify(Qd, Rd, labd, k)), args.steps, args.warmup)
    log(f"[bench] classify {n} x {m} x {d} (k = {k}, {p['comps']} classes): {sec * 1e3:.4f} ms, "
        f"{n * m / sec:.4e} pairs/s")
    result = {"metric": "query-ref pairs/sec", "value": float(n) * m / sec, "unit": "pairs/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "classify_gmm16384_d96", "n": n, "m": m, "d": d, "k": k, "classes": p["comps"]},
              "kernels": kernels}
    if not args.no_cpu_baseline:
        from oracle import classify as C

        t0 = time.perf_counter()
        ref = C.classify(Q, R, lab, k, threads=host_threads())
        cpu_s = time.perf_counter() - t0
        agree = float(np.mean(out[0].cpu().numpy() == ref))
        result["cpu_baseline"] = {"value": float(n) * m / cpu_s, "unit": "pairs/s", "cores": host_threads(),
                                  "kind": "oracle", "sample": f"all {n} queries (FP64), {cpu_s:.2f} s"}
        result["parity_vs_oracle"] = {"agreement": agree}
        log(f"[bench] agreement with the oracle's votes: {agree:.6f}")
    return result


# ------------------------------------------------------------- timing table
def bench_table(args):
    """The timing table of the paper's experiments, reshaped for this GPU:
    N query and N reference points (uniform [0,1) floats, seeded), D dims,
    k = 20, Euclidean, for N in 1200 .. 38400 and D in 8 .. 96.  Each cell is
    timed end to end (inputs in pinned host memory copied in, results copied
    back) and device-resident, over a few repetitions."""
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    Ns = [1200, 2400, 4800, 9600, 19200, 38400]
    Ds = [8, 16, 32, 64, 80, 96]
    k, reps = 20, max(3, args.steps)
    cells = []
    for D in Ds:
        for N in Ns:
            R = synthdata.uniform((N, D), 1000 + D, 0)
            Q = synthdata.uniform((N, D), 1000 + D, 1)
            Rh, Qh = torch.from_numpy(R).pin_memory(), torch.from_numpy(Q).pin_memory()
            dh = torch.empty((N, k), dtype=torch.float32).pin_memory()
            ih = torch.empty((N, k), dtype=torch.int32).pin_memory()
            Rd, Qd = Rh.cuda(), Qh.cuda()

            def e2e():
                Rx = Rh.to("cuda", non_blocking=True)
                Qx = Qh.to("cuda", non_blocking=True)
                dist, idx = K.search(Qx, Rx, k, "l2")
                dh.copy_(dist, non_blocking=True)
                ih.copy_(idx, non_blocking=True)

            times = {}
            for name, fn in (("end_to_end", e2e), ("resident", lambda: K.search(Qd, Rd, k, "l2"))):
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn()
                torch.cuda.synchronize()
                times[name] = (time.perf_counter() - t0) / reps
            cells.append({"N": N, "D": D, "end_to_end_ms": times["end_to_end"] * 1e3,
                          "resident_ms": times["resident"] * 1e3})
            log(f"[bench] D={D:3d} N={N:6d}: end to end {times['end_to_end'] * 1e3:8.3f} ms, "
                f"resident {times['resident'] * 1e3:8.3f} ms")
    big = [c for c in cells if c["N"] == Ns[-1] and c["D"] == Ds[-1]][0]
    return {"metric": "query-ref pairs/sec", "value": float(Ns[-1]) ** 2 / (big["resident_ms"] / 1e3),
            "unit": "pairs/s", "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": big["resident_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "table_uniform", "N": Ns, "D": Ds, "k": k, "distance": "l2"}, "cells": cells}


def bench_copy(args):
    import torch

    nbytes = 1 << 30
    src = torch.rand(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    sec, _ = timed(__import__("paper_0804_1448_amd"), torch, lambda: dst.copy_(src), args.steps, args.warmup)
    gbs = 2.0 * nbytes / sec / 1e9
    log(f"[bench] copy {nbytes} bytes: {sec * 1e3:.3f} ms, {gbs:.1f} GB/s (read + write)")
    return {"metric": "device copy bandwidth", "value": gbs, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "copy1g", "bytes_read": nbytes, "bytes_written": nbytes},
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS, "traffic": None}}


def bench_peaks(args):
    """Measured issue rates of the instructions the roofline peaks assume:
    the Manhattan kernel's vector subtract (DPP operand) + absolute add, the
    BF16 32x32x16 and float32 32x32x2 matrix instructions, and 16-byte LDS
    reads; each with the shader clock of the run (s_memtime against the
    100 MHz s_memrealtime)."""
    import ctypes

    import torch

    import paper_0804_1448_amd.build as B

    lib = ctypes.CDLL(B.PEAKS_LIB)
    lib.knn_peak_launch.restype = ctypes.c_int
    lib.knn_peak_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    # (name, which, workgroups of 4 waves, iterations, work per wave and iteration, unit, datasheet peak)
    cases = [("valu_sub_dpp_absadd", 0, cus * 8, 20000, 64 * 16, "T lane-ops/s", PEAK_VALU_TOPS),
             ("mfma_bf16_32x32x16", 1, cus * 8, 10000, 8 * 32768, "TFLOP/s", PEAK_BF16_MFMA_TFLOPS),
             ("mfma_f32_32x32x2", 2, cus * 8, 10000, 8 * 4096, "TFLOP/s", PEAK_FP32_MFMA_TFLOPS),
             ("lds_read_b128", 3, cus * 4, 20000, 8 * 1024, "TB/s", PEAK_LDS_TBS)]
    stream = torch.cuda.current_stream()
    out = {}
    for name, which, blocks, iters, per_wave, unit, peak in cases:
        buf = torch.empty(blocks * 256, device="cuda")
        clk = torch.zeros(4, dtype=torch.int64, device="cuda")
        launch = lambda: lib.knn_peak_launch(which, blocks, iters, ctypes.c_void_p(buf.data_ptr()),
                                             ctypes.c_void_p(clk.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
        for _ in range(args.warmup):
            if launch() != 0:
                raise RuntimeError(f"peak kernel {name} launch failed")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            launch()
        ev1.record(stream)
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) / 1e3 / args.steps
        c = clk.cpu().tolist()
        ghz = (c[2] - c[0]) / ((c[3] - c[1]) / 100e6) / 1e9 if c[3] > c[1] else float("nan")
        work = float(blocks) * 4 * iters * per_wave
        rate = work / sec / 1e12
        per_cu_clk = work / sec / (cus * ghz * 1e9)
        out[name] = {"rate": rate, "unit": unit, "datasheet_peak": peak, "frac_of_datasheet": rate / peak,
                     "clock_ghz": ghz, "per_cu_per_clock": per_cu_clk, "peak_at_2p4ghz": per_cu_clk * cus * 2.4e9 / 1e12,
                     "ms": sec * 1e3}
        log(f"[bench] {name}: {rate:.2f} {unit} ({rate / peak:.3f} of {peak:.1f}) at {ghz:.3f} GHz, "
            f"{per_cu_clk:.1f} per CU per clock")
    # BF16 matrix rate by independent accumulator chains per wave and waves per SIMD
    lib.knn_peak_launch_chains.restype = ctypes.c_int
    lib.knn_peak_launch_chains.argtypes = lib.knn_peak_launch.argtypes
    chains = {}
    for ch in (1, 2, 4, 8):
        for wps in (1, 2, 4, 8):
            blocks, iters = cus * wps, 8192 // ch
            buf = torch.empty(blocks * 256, device="cuda")
            clk = torch.zeros(4, dtype=torch.int64, device="cuda")
            launch = lambda: lib.knn_peak_launch_chains(ch, blocks, iters, ctypes.c_void_p(buf.data_ptr()),
                                                        ctypes.c_void_p(clk.data_ptr()),
                                                        ctypes.c_void_p(stream.cuda_stream))
            if launch() != 0:
                raise RuntimeError("peak chains kernel launch failed")
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(3):
                launch()
            ev1.record(stream)
            torch.cuda.synchronize()
            sec = ev0.elapsed_time(ev1) / 3e3
            chains[f"chains{ch}_waves{wps}"] = float(blocks) * 4 * iters * ch * 32768 / sec / 1e12
        log(f"[bench] bf16 MFMA, {ch} chains per wave, 1/2/4/8 waves per SIMD: "
            + " / ".join(f"{chains[f'chains{ch}_waves{w}']:.0f}" for w in (1, 2, 4, 8)) + " TFLOP/s")
    out["mfma_bf16_by_chains_and_waves_tflops"] = chains
    return {"metric": "measured peak issue rates", "value": out["mfma_bf16_32x32x16"]["rate"], "unit": "TFLOP/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "bf16/f32", "data": "synthetic", "config": {"workload": "peaks", "cus": cus},
            "peaks": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--mode", default="precision", choices=["pairs", "precision", "batched", "serve", "copy", "entropy",
                                                      "mahalanobis", "classify", "table", "peaks"])
    ap.add_argument("--workload", default="gmm16384_d96", choices=sorted(WORKLOAD_METRICS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target host time of the oracle sample")
    ap.add_argument("--recall-queries", type=int, default=2048,
                    help="precision mode: seeded queries checked against the FP64 oracle (recall@k sample)")
    ap.add_argument("--instances", type=int, default=512, help="batched mode: number of instances")
    ap.add_argument("--batch-extra", type=int, default=28,
                    help="batched mode: extra candidates re-ranked per query (k + extra <= 128 keeps every instance, "
                         "k up to 100, in the one launch of the 32x32-tile kernel)")
    ap.add_argument("--requests", type=int, default=10000, help="serve mode: requests per trace")
    ap.add_argument("--sizes", default="uniform", choices=["uniform", "loguniform"],
                    help="serve mode: request size distribution")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 0.8], help="serve mode: fractions of capacity")
    ap.add_argument("--serve-mem", type=int, default=8, help="serve mode: request memory budget, GiB")
    ap.add_argument("--serve-streams", type=int, default=2, help="serve mode: batches in flight (one stream each)")
    ap.add_argument("--serve-one-set", action="store_true",
                    help="serve mode: batch requests of one set only (16-bit sets otherwise share launches)")
    ap.add_argument("--serve-extra", type=int, default=14,
                    help="serve mode: extra candidates re-ranked per query (k + extra <= 64 keeps every request "
                         "on the 32x32-tile kernel for k <= 50)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this path does not shard "
              "across GPUs in this build)", file=sys.stderr)
        sys.exit(2)
    defaults = {"pairs": (50, 5), "precision": (10, 2), "batched": (10, 2), "serve": (0, 0), "copy": (20, 3), "entropy": (20, 3), "mahalanobis": (20, 3), "classify": (20, 3), "table": (5, 1), "peaks": (5, 1)}
    if args.steps is None:
        args.steps = defaults[args.mode][0]
    if args.warmup is None:
        args.warmup = defaults[args.mode][1]

    import torch

    import paper_0804_1448_amd as K

    K.load()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    fn = {"pairs": bench_pairs, "precision": bench_precision, "batched": bench_batched, "serve": bench_serve,
          "copy": bench_copy, "entropy": bench_entropy, "mahalanobis": bench_mahalanobis,
          "classify": bench_classify, "table": bench_table, "peaks": bench_peaks}
    print(json.dumps(fn[args.mode](args)), flush=True)


if __name__ == "__main__":
    main()
