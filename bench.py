#!/usr/bin/env python3
"""Benchmark of the brute-force k-NN path on one MI355X.

A step is one pass of the whole path over the workload: for each distance of
the workload, knn_search (reference preparation, query preparation, fused
distance tiles + per-query selection, slice merge, exact re-rank and output)
on float32 inputs already resident in device memory.  The default workload
is 16384 references and 16384 queries in 96 dimensions from a 64-component
Gaussian mixture, k = 20, searched with the Euclidean distance (matrix cores)
and the Manhattan distance (vector ALUs).

Prints one JSON line.  Besides the throughput it reports the roofline of the
dominant kernel (its average duration measured with HIP events on the stream
it runs on) and the FP64 oracle timed on the host cores over a query sample,
which also checks the GPU result on that sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# peaks of one MI355X (vendor figures)
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2516.6
# vector ALU, one non-packed lane operation per lane per clock:
# 256 CUs x 64 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0

WORKLOAD_METRICS = {
    "gmm16384_d96": ["l2", "l1"],
    "uniform4096_d32": ["l2", "l1"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_roofline(name: str, avg_s: float, n: int, m: int, d: int):
    """Algorithmic work of one fused launch over n x m pairs, against its peak."""
    if name.startswith("fused_l2"):
        flops = 2.0 * d * n * m  # cross term q.r: d multiply-adds per pair
        peak = PEAK_FP32_MFMA_TFLOPS if name.endswith("f32") else PEAK_BF16_MFMA_TFLOPS
        ach = flops / avg_s / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": None, "kernel": name, "avg_ms": avg_s * 1e3, "work_per_launch": flops}
    ops = 2.0 * d * n * m  # one subtract + one absolute accumulate (sum or max) per pair and dimension
    ach = ops / avg_s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TFLOP/s", "frac": ach / PEAK_VALU_TOPS,
            "traffic": None, "kernel": name, "avg_ms": avg_s * 1e3, "work_per_launch": ops}


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="gmm16384_d96", choices=sorted(WORKLOAD_METRICS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target host time of the oracle sample")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this path does not shard "
              "across GPUs in this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0804_1448_amd as K
    import synthdata

    K.load()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
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
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    K.timing.reset()
    K.timing.enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    K.timing.enable(False)
    kern = K.timing.all()
    ms_per_step = (t1 - t0) / args.steps * 1e3
    pairs_per_step = float(n) * m * len(metrics)
    value = pairs_per_step / (ms_per_step / 1e3)
    log(f"[bench] {args.steps} steps: {ms_per_step:.4f} ms/step, {value:.4e} pairs/s")
    kernels = {name: {"avg_ms": tot / cnt, "launches": cnt, "total_ms": tot} for name, (tot, cnt) in kern.items()}
    for name, v in kernels.items():
        log(f"[bench]   {name:16s} avg {v['avg_ms']:.4f} ms x {v['launches']}")

    rooflines = {}
    for name, v in kernels.items():
        if name.startswith("fused_"):
            rooflines[name] = kernel_roofline(name, v["avg_ms"] / 1e3, n, m, d)
    dominant = max(rooflines, key=lambda nm: kernels[nm]["total_ms"])
    roof = dict(rooflines[dominant])

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
        "roofline": roof,
        "rooflines": rooflines,
        "kernels": kernels,
    }

    if not args.no_cpu_baseline:
        import oracle
        from oracle.check import compare

        threads = host_threads()
        rng = np.random.default_rng(12345)
        # calibrate: time a small sample, then size the sample to the target host time
        probe = rng.choice(n, size=min(n, 16), replace=False)
        tp = time.perf_counter()
        for mt in metrics:
            oracle.knn(Q[probe], R, k, mt, threads=threads)
        per_query = (time.perf_counter() - tp) / len(probe)
        nsamp = int(min(n, max(len(probe), args.cpu_seconds / max(per_query, 1e-9))))
        rows = np.sort(rng.choice(n, size=nsamp, replace=False))
        log(f"[bench] oracle sample: {nsamp} queries x {m} references x {len(metrics)} distances, {threads} threads")
        tc = time.perf_counter()
        refs = {mt: oracle.knn(Q[rows], R, k, mt, threads=threads) for mt in metrics}
        cpu_s = time.perf_counter() - tc
        cpu_value = float(nsamp) * m * len(metrics) / cpu_s
        parity = {}
        for mt in metrics:
            dist = outs[mt][0].cpu().numpy()
            idx = outs[mt][1].cpu().numpy()
            rep = compare(Q, R, k, mt, dist, idx, tol=1e-5, ref=refs[mt], rows=rows)
            parity[mt] = {kk: rep[kk] for kk in ("ok", "max_rel_err", "recall", "recall_tie", "bad_dist", "bad_idx",
                                                   "queries")}
        result["cpu_baseline"] = {
            "value": cpu_value, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{nsamp} seeded queries of {n} against all {m} references, distances {metrics}, "
                      f"FP64 brute force (select mode), {cpu_s:.2f} s",
        }
        result["parity_vs_oracle"] = parity
        result["recall_at_k"] = {mt: parity[mt]["recall"] for mt in metrics}

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
