"""Seeded synthetic point sets shared by the tests, the benchmark and the oracle runs.

This module only draws numbers: it holds none of the k-NN arithmetic (no
distances, no selection, no rounding to a compute precision).  The paper states
neither a data distribution nor a dataset for its timing table ("typical
values", Section 3), so every workload is one of the synthetic recipes below:

* ``uniform(shape)``: i.i.d. uniform [0, 1) in float32 (numpy's float32 path,
  i.e. multiples of 2**-24).
* ``gmm(n, d, comps, sigma)``: an isotropic Gaussian mixture; centres uniform in
  [0, 1)^d, equal component weights, point = centre + sigma * N(0, I) drawn in
  float64 and rounded once to float32.  References and queries are drawn from
  the same mixture with different streams.

Seeds come from ``numpy.random.SeedSequence([workload_id, role])`` so that every
consumer regenerates bit-identical arrays.  Roles: 0 references, 1 queries,
2 mixture centres, 3 request stream, 4 and up for anything else a workload
needs.
"""
from __future__ import annotations

import numpy as np

ROLE_REFS = 0
ROLE_QUERIES = 1
ROLE_CENTRES = 2
ROLE_REQUESTS = 3
ROLE_EXTRA = 4
GMM_BLOCK = 4096


def rng_for(workload_id: int, role: int) -> np.random.Generator:
    """PCG64 generator for one (workload, role) stream."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(workload_id), int(role)])))


def uniform(shape, workload_id: int, role: int) -> np.ndarray:
    """i.i.d. U[0,1) float32 array of ``shape``."""
    return rng_for(workload_id, role).random(shape, dtype=np.float32)


def gmm_centres(comps: int, d: int, workload_id: int) -> np.ndarray:
    """Mixture centres, uniform in [0,1)^d, float64."""
    return rng_for(workload_id, ROLE_CENTRES).random((comps, d))


def gmm(npts: int, d: int, comps: int, sigma: float, workload_id: int, role: int,
        return_labels: bool = False, threads: int = 1, centres_id: int | None = None):
    """``npts`` float32 points from the isotropic mixture of workload ``workload_id``.

    Points are drawn in blocks of ``GMM_BLOCK`` from per-block streams
    (``SeedSequence([workload_id, role, block])``), so a shorter set is an
    exact prefix of a longer one and a million-point set never needs a float64
    copy of the whole array.  Blocks are independent, so ``threads`` > 1
    fills them concurrently with identical results.  ``centres_id`` takes the
    mixture centres of another workload id (several sets of one mixture).
    """
    centres = gmm_centres(comps, d, workload_id if centres_id is None else centres_id)
    out = np.empty((npts, d), dtype=np.float32)
    labels = np.empty(npts, dtype=np.int32) if return_labels else None

    def fill(b):
        s = b * GMM_BLOCK
        e = min(npts, s + GMM_BLOCK)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(workload_id), int(role), b])))
        lab = rng.integers(0, comps, GMM_BLOCK)[: e - s]
        noise = rng.standard_normal((GMM_BLOCK, d))[: e - s]
        out[s:e] = (centres[lab] + sigma * noise).astype(np.float32)
        if return_labels:
            labels[s:e] = lab

    nblocks = (npts + GMM_BLOCK - 1) // GMM_BLOCK
    if threads > 1 and nblocks > 1:
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(fill, range(nblocks)))
    else:
        for b in range(nblocks):
            fill(b)
    if return_labels:
        return out, labels
    return out


def integer_grid(shape, lo: int, hi: int, workload_id: int, role: int) -> np.ndarray:
    """Integers in [lo, hi) as float32: exact in every precision, many exact ties."""
    return rng_for(workload_id, role).integers(lo, hi, shape).astype(np.float32)


def dyadic(shape, bits: int, workload_id: int, role: int) -> np.ndarray:
    """Values j / 2**bits, j uniform in [-2**bits, 2**bits), as float32 (exact)."""
    j = rng_for(workload_id, role).integers(-(1 << bits), 1 << bits, shape)
    return (j.astype(np.float64) / float(1 << bits)).astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads.  Each returns (R, Q) float32 arrays plus its parameters.
# ---------------------------------------------------------------------------

WORKLOADS = {
    # small uniform case: m = n = 4096, d = 32, k = 20
    "uniform4096_d32": dict(wid=1, m=4096, n=4096, d=32, k=20, kind="uniform"),
    # paper-scale brute force: m = n = 16384, d = 96, k = 20, 64-component mixture
    "gmm16384_d96": dict(wid=2, m=16384, n=16384, d=96, k=20, kind="gmm", comps=64, sigma=0.05),
    # precision form: m = 2**20, n = 65536, d = 128, k = 32, 1024 components
    "gmm1m_d128": dict(wid=3, m=1 << 20, n=65536, d=128, k=32, kind="gmm", comps=1024, sigma=0.1),
}

# batched form: 512 independent instances, uniform [0,1) data
BATCH512 = dict(wid=7, count=512, m=(1000, 200000), n=(16, 4096), d=(16, 32, 64, 128), k=(1, 8, 32, 100))

# serving form: four resident sets of one 1024-component mixture (sigma 0.1,
# d = 128) with 1, 2, 3 and 4 Mi points; requests of 1..2048 queries
# (uniform; log-uniform as a variant), k in {10, 50}, set uniform, Poisson
# arrivals
SERVE4 = dict(wid=6, sets=(1 << 20, 2 << 20, 3 << 20, 4 << 20), d=128, comps=1024, sigma=0.1,
              n=(1, 2048), k=(10, 50), pool=16384)


def batch_specs(spec=BATCH512, count: int | None = None):
    """[(m, n, d, k)] of the batched workload (k <= m always holds: m >= 1000)."""
    rng = rng_for(spec["wid"], ROLE_EXTRA)
    cnt = spec["count"] if count is None else count
    out = []
    for _ in range(cnt):
        m = int(rng.integers(spec["m"][0], spec["m"][1] + 1))
        n = int(rng.integers(spec["n"][0], spec["n"][1] + 1))
        d = int(rng.choice(spec["d"]))
        k = int(rng.choice(spec["k"]))
        out.append((m, n, d, min(k, m)))
    return out


def batch_instance(i: int, m: int, n: int, d: int, spec=BATCH512):
    """(R, Q) of instance ``i`` of the batched workload."""
    R = rng_for(spec["wid"] * 100000 + i, ROLE_REFS).random((m, d), dtype=np.float32)
    Q = rng_for(spec["wid"] * 100000 + i, ROLE_QUERIES).random((n, d), dtype=np.float32)
    return R, Q


def serve_set(j: int, spec=SERVE4, m: int | None = None, threads: int = 1) -> np.ndarray:
    """Reference set ``j`` of the serving workload (a prefix of ``m`` rows if given)."""
    mm = spec["sets"][j] if m is None else m
    return gmm(mm, spec["d"], spec["comps"], spec["sigma"], spec["wid"] * 100 + j, ROLE_REFS, threads=threads,
               centres_id=spec["wid"])


def serve_queries(j: int, spec=SERVE4, count: int | None = None) -> np.ndarray:
    """Query pool of set ``j``: points of the same mixture, another stream."""
    return gmm(spec["pool"] if count is None else count, spec["d"], spec["comps"], spec["sigma"],
               spec["wid"] * 100 + j, ROLE_QUERIES, centres_id=spec["wid"])


def serve_requests(count: int, spec=SERVE4, seed_role: int = ROLE_REQUESTS, sizes: str = "uniform"):
    """[(gap, set, offset, n, k)]: exponential gaps of unit mean (scale by 1/rate),
    set index, offset into that set's query pool, size and k.  ``sizes`` is
    "uniform" (n uniform in the range) or "loguniform"."""
    rng = rng_for(spec["wid"], seed_role)
    lo, hi = spec["n"]
    out = []
    for _ in range(count):
        gap = float(rng.exponential(1.0))
        s = int(rng.integers(len(spec["sets"])))
        if sizes == "uniform":
            n = int(rng.integers(lo, hi + 1))
        else:
            n = int(min(hi, max(lo, np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1)))))))
        off = int(rng.integers(0, spec["pool"] - n + 1))
        k = int(rng.choice(spec["k"]))
        out.append((gap, s, off, n, k))
    return out


def workload(name: str, n: int | None = None, m: int | None = None):
    """Return (R, Q, params) for a named workload; ``n``/``m`` cut a prefix."""
    p = dict(WORKLOADS[name])
    mm = p["m"] if m is None else m
    nn = p["n"] if n is None else n
    if p["kind"] == "uniform":
        R = uniform((p["m"], p["d"]), p["wid"], ROLE_REFS)[:mm]
        Q = uniform((p["n"], p["d"]), p["wid"], ROLE_QUERIES)[:nn]
    else:
        R = gmm(mm, p["d"], p["comps"], p["sigma"], p["wid"], ROLE_REFS)
        Q = gmm(nn, p["d"], p["comps"], p["sigma"], p["wid"], ROLE_QUERIES)
    p["m"], p["n"] = mm, nn
    return np.ascontiguousarray(R), np.ascontiguousarray(Q), p
