"""Tie-aware comparison of a k-NN result with the FP64 oracle.

TEST INFRASTRUCTURE ONLY (used by the tests and the benchmark's CPU baseline).

For query i, D*[i, r] is the oracle's r-th smallest distance and tol the
relative tolerance.  A result (dist, idx) passes when, for every rank r < k:

* distances (T1):  |dist[i,r] - D*[i,r]| <= tol * D*[i,r];
* indices (T2):    the k indices of a row are distinct and in [0, m), and the
  oracle distance of the returned reference, D64(q_i, r_idx[i,r]), lies within
  tol * D*[i,r] of D*[i,r].  The returned index therefore equals the oracle's
  one unless another reference is within the tolerance at that rank: that
  allows reorderings inside near-tie groups and swaps across the k boundary,
  and nothing else;
* pairing:         the returned distance is the distance to the returned
  reference: |dist[i,r] - D64(q_i, r_idx[i,r])| <= tol * D64(q_i, r_idx[i,r]).
  For the float32 path it follows from T1 and T2 up to a factor 2; for the
  low-precision forms, where T1 binds only the hits, it is what ties every
  returned distance (hit or miss) to its index.

Recall for the low-precision forms:
* strict recall@k = mean_i |S_i intersect S*_i| / k (S* = oracle's top-k index set);
* tie-aware recall = fraction of returned references whose oracle distance is
  <= D*[i,k-1] * (1 + tol).
"""
from __future__ import annotations

import numpy as np

from . import knn, pair_dist


def compare(Q, R, k, metric, dist, idx, tol=1e-5, ref=None, rows=None):
    """Return a report dict; ``ref`` = precomputed oracle (D*, I*) for ``rows``.

    ``rows`` selects the query rows (of Q, dist and idx) to check; default all.
    """
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    R = np.ascontiguousarray(R, dtype=np.float32)
    dist = np.asarray(dist)
    idx = np.asarray(idx).astype(np.int64)
    if rows is None:
        rows = np.arange(Q.shape[0])
    rows = np.asarray(rows, dtype=np.int64)
    dist = dist[rows].astype(np.float64)
    idx = idx[rows]
    if ref is None:
        ref = knn(Q[rows], R, k, metric)
    Ds, Is = ref
    if Ds.shape != (rows.size, k) or Is.shape != (rows.size, k) or dist.shape != (rows.size, k):
        raise ValueError(f"shapes differ: oracle {Ds.shape}, result {dist.shape}, {rows.size} rows x k = {k}")
    m = R.shape[0]
    nq = rows.size
    rep = {"queries": int(nq), "k": int(k), "tol": tol}
    in_range = (idx >= 0) & (idx < m)
    srt = np.sort(np.where(in_range, idx, -1 - np.arange(k)[None, :]), axis=1)
    distinct = np.all(srt[:, 1:] != srt[:, :-1], axis=1) if k > 1 else np.ones(nq, bool)
    rep["bad_index_rows"] = int(np.sum(~(np.all(in_range, axis=1) & distinct)))
    safe_idx = np.where(in_range, idx, 0)
    d64 = pair_dist(Q, R, np.repeat(rows, k), safe_idx.ravel(), metric).reshape(nq, k)
    lim = tol * Ds
    bad_dist = ~(np.abs(dist - Ds) <= lim)  # NaN fails
    bad_idx = (np.abs(d64 - Ds) > lim) | ~in_range
    bad_pair = ~(np.abs(dist - d64) <= tol * d64) | ~in_range
    rep["bad_dist"] = int(bad_dist.sum())
    rep["bad_idx"] = int(bad_idx.sum())
    rep["bad_pair"] = int(bad_pair.sum())
    pos = Ds > 0
    rel = np.zeros_like(Ds)
    rel[pos] = np.abs(dist[pos] - Ds[pos]) / Ds[pos]
    rel[~pos] = np.where(dist[~pos] == 0, 0.0, np.inf)
    rep["max_rel_err"] = float(rel.max()) if rel.size else 0.0
    hits = np.zeros_like(idx, dtype=bool)
    for i in range(nq):
        hits[i] = np.isin(idx[i], Is[i])
    rep["recall"] = float(hits.sum() / max(1, nq * k))
    kth = Ds[:, -1:] * (1 + tol)
    rep["recall_tie"] = float(np.sum((d64 <= kth) & in_range) / max(1, nq * k))
    relh = np.zeros_like(d64)
    posh = d64 > 0
    relh[posh] = np.abs(dist[posh] - d64[posh]) / d64[posh]
    relh[~posh] = np.where(dist[~posh] == 0, 0.0, np.inf)
    rep["max_rel_err_hits"] = float(relh[hits].max()) if hits.any() else 0.0
    rep["max_rel_err_pair"] = float(relh.max()) if relh.size else 0.0
    rep["exact_idx_match"] = float(np.mean(idx == Is))
    rep["ok"] = (rep["bad_index_rows"] == 0 and rep["bad_dist"] == 0 and rep["bad_idx"] == 0
                 and rep["bad_pair"] == 0)
    return rep


def recall_ci(recall: float, trials: int, z: float = 1.96):
    """Wilson score interval for a recall estimated from ``trials`` slots."""
    if trials <= 0:
        return (0.0, 1.0)
    p = recall
    den = 1 + z * z / trials
    centre = (p + z * z / (2 * trials)) / den
    half = z * np.sqrt(p * (1 - p) / trials + z * z / (4 * trials * trials)) / den
    return (float(max(0.0, centre - half)), float(min(1.0, centre + half)))
