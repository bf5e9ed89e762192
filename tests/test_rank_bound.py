"""The bound behind the rank slots of the 32x32 kernel, checked on the CPU.

A query's references are split over P slices (the split-m brute force of
Section 2.1).  Each slice publishes the score of its r-th best key so far,
r = max(ceil(k'/P), ceil(k'/64)); any g = ceil(k'/r) slices hold at least
g * r >= k' keys at or below the largest of their published values, so that
largest value is never below the query's k'-th best score over the whole set,
and the kernel may drop every score above it.  A slice's r-th best only falls
as it sees more keys, so a value read late (stale) is larger and still a bound.
These tests check the inequality on random and clustered scores, for the
group sizes and ranks the library chooses, at every prefix of the scan."""
import math

import numpy as np
import pytest


def rank_plan(kc, P):
    r = max(math.ceil(kc / P), math.ceil(kc / 64))
    g = math.ceil(kc / r)
    G = max(1, min(P // g, 4))
    return r, g, G


@pytest.mark.parametrize("kc,P", [(24, 8), (64, 8), (64, 64), (64, 256), (29, 100), (122, 16), (128, 9), (1, 8)])
def test_plan_groups_hold_k_prime_keys(kc, P):
    r, g, G = rank_plan(kc, P)
    assert g * r >= kc          # a group's published values stand for at least k' keys
    assert g <= P and g <= 64   # a group fits the query's slices and two lane halves of 32
    assert r <= 64              # the r-th key lies in the first 64 of a list
    assert 1 <= G and G * g <= P


@pytest.mark.parametrize("seed,kc,P,clustered", [(1, 64, 64, False), (2, 64, 256, True), (3, 24, 8, True),
                                                 (4, 122, 16, False), (5, 29, 100, True)])
def test_group_maximum_bounds_the_union_kth(seed, kc, P, clustered):
    rng = np.random.default_rng(seed)
    L = 512  # references per slice
    if clustered:  # a few close references among many far ones, as a query's own cluster
        s = rng.normal(10.0, 1.0, (P, L))
        near = rng.random((P, L)) < 0.01
        s[near] = rng.normal(0.0, 1.0, near.sum())
    else:
        s = rng.random((P, L))
    r, g, G = rank_plan(kc, P)
    for t in (r, 2 * r, L // 4, L):  # prefixes of every slice's scan
        seen = np.sort(s[:, :t], axis=1)
        published = seen[:, r - 1]                    # each slice's r-th best so far
        kth_all = np.sort(s.ravel())[kc - 1]          # the query's k'-th best over the whole set
        groups = [published[i * g:(i + 1) * g] for i in range(G)]
        bound = min(grp.max() for grp in groups)
        assert bound >= kth_all
        # every one of the k' best over the whole set survives the filter
        assert np.sort(s.ravel())[:kc].max() <= bound
    # a stale value (an earlier prefix) is never below a later one
    early = np.sort(s[:, :r], axis=1)[:, r - 1]
    late = np.sort(s, axis=1)[:, r - 1]
    assert np.all(early >= late)
