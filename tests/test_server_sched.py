"""Scheduler tests of the serving engine in dry-run mode (no device work).

In a dry run a batch takes ``us_per_query * queries`` microseconds and
writes, for every query of every request in it, dist = the set index and
idx = the batch's launch sequence number, so routing, batching, memory
admission and queue order are visible from the results alone.
"""
from __future__ import annotations

import time

import numpy as np
import pytest


@pytest.fixture(scope="module")
def K():
    import paper_0804_1448_amd as K
    import paper_0804_1448_amd._lib as L

    if not __import__("os").path.exists(L.LIB_PATH):
        import paper_0804_1448_amd.build as B

        B.build()
    return K


D = 8


def q(n, seed=0):
    return np.random.default_rng(seed).random((n, D), dtype=np.float32)


def wait_all(srv, tickets):
    return {t: srv.wait(t) for t in tickets}


def test_routing_and_results_shape(K):
    with K.Server.dry(3, m=1000, d=D, us_per_query=1.0) as srv:
        subs = []
        for i in range(30):
            s, n, k = i % 3, 1 + (i * 7) % 13, 1 + i % 5
            subs.append((srv.submit(s, q(n, i), k), s, n, k))
        for t, s, n, k in subs:
            dist, idx, lat = srv.wait(t)
            assert dist.shape == (n, k) and idx.shape == (n, k)
            assert np.all(dist == s)
            assert np.all(idx == idx[0, 0])
            assert lat > 0
        st = srv.stats()
        assert st["submitted"] == st["completed"] == 30
        assert st["queries"] == sum(n for _, _, n, _ in subs)


def test_batch_mates_share_set_and_respect_max_queries(K):
    maxq = 40
    with K.Server.dry(2, m=500, d=D, us_per_query=200.0, max_batches=1, max_batch_queries=maxq) as srv:
        # the first request occupies the only stream; the rest queue up behind it
        subs = [(srv.submit(0, q(5), 3), 0, 5, 3)]
        rng = np.random.default_rng(3)
        for i in range(60):
            s, k, n = int(rng.integers(2)), int(rng.choice([3, 4])), int(rng.integers(1, 15))
            subs.append((srv.submit(s, q(n, i), k), s, n, k))
        res = wait_all(srv, [t for t, *_ in subs])
        by_batch = {}
        for t, s, n, k in subs:
            by_batch.setdefault(int(res[t][1][0, 0]), []).append((s, n, k))
        mixed_k = 0
        for b, members in by_batch.items():
            assert len({s for s, _, _ in members}) == 1, (b, members)
            assert sum(n for _, n, _ in members) <= maxq
            mixed_k += len({k for _, _, k in members}) > 1
        # queued requests were batched: far fewer launches than requests, and
        # requests of different k share launches
        assert len(by_batch) < len(subs) / 3
        assert mixed_k > 0
        assert srv.stats()["batches"] == len(by_batch)


def test_16bit_batches_take_every_set(K):
    """16-bit servers put waiting requests of every set (k + s <= 128) into one
    launch; k + s > 128 requests, and every request with one_set=True, batch
    with their own set only.  Each request's dist reads its own set."""
    with K.Server.dry(3, m=5000, d=D, us_per_query=200.0, max_batches=1, max_batch_queries=200,
                      precision="fp16") as srv:
        first = srv.submit(0, q(5), 3)  # occupies the only stream
        rng = np.random.default_rng(7)
        subs = []
        for i in range(40):
            s, k, n = int(rng.integers(3)), int(rng.choice([3, 50, 100])), int(rng.integers(1, 9))
            subs.append((srv.submit(s, q(n, i), k), s, n, k))
        res = wait_all(srv, [first] + [t for t, *_ in subs])
        by_batch = {}
        for t, s, n, k in subs:
            assert np.all(res[t][0] == s)
            by_batch.setdefault(int(res[t][1][0, 0]), []).append((s, n, k))
        mixed = 0
        for members in by_batch.values():
            big = [k for _, _, k in members if k + 32 > 128]
            assert not big or len({s for s, _, _ in members}) == 1, members  # k' > 128: a batch of one set
            mixed += len({s for s, _, _ in members}) > 1
        assert mixed > 0, "no batch mixed sets"
    with K.Server.dry(3, m=5000, d=D, us_per_query=200.0, max_batches=1, max_batch_queries=200,
                      precision="fp16", one_set=True) as srv:
        first = srv.submit(0, q(5), 3)
        subs = [(srv.submit(i % 3, q(4, i), 3), i % 3) for i in range(30)]
        res = wait_all(srv, [first] + [t for t, _ in subs])
        by_batch = {}
        for t, s in subs:
            by_batch.setdefault(int(res[t][1][0, 0]), set()).add(s)
        assert all(len(v) == 1 for v in by_batch.values())


def test_fifo_head_no_starvation(K):
    """With one stream and no batching possible, requests complete in arrival order."""
    with K.Server.dry(2, m=500, d=D, us_per_query=50.0, max_batches=1, max_batch_queries=8) as srv:
        subs = [srv.submit(i % 2, q(8, i), 2) for i in range(40)]
        seqs = [int(srv.wait(t)[1][0, 0]) for t in subs]
        assert seqs == sorted(seqs)
        assert len(set(seqs)) == len(seqs)


def test_other_set_is_not_starved_by_a_stream_of_mates(K):
    """A request of set 1 behind many set-0 requests launches once it heads the queue."""
    with K.Server.dry(2, m=500, d=D, us_per_query=100.0, max_batches=1, max_batch_queries=16) as srv:
        first = [srv.submit(0, q(8, i), 2) for i in range(4)]
        lone = srv.submit(1, q(8), 2)
        later = [srv.submit(0, q(8, 100 + i), 2) for i in range(20)]
        res = wait_all(srv, first + [lone] + later)
        b_lone = int(res[lone][1][0, 0])
        b_first = max(int(res[t][1][0, 0]) for t in first)
        # set-0 requests after it may join the batches of earlier set-0 heads,
        # but the lone request launches right after the batches its
        # predecessors head; at most the first four requests' batches precede it
        assert b_lone <= b_first + 1
        assert b_lone <= 4


def test_small_request_passes_a_head_waiting_for_memory(K):
    """A request too large for the memory left waits; a later small one that
    fits launches meanwhile (for at most 50 ms of the large one's wait)."""
    probe = K.Server.dry(1, m=2000, d=D, us_per_query=0.0, mem_budget=1 << 40)
    probe.wait(probe.submit(0, q(200), 16))
    one = probe.stats()["peak_mem_in_flight"]
    probe.close()
    with K.Server.dry(2, m=2000, d=D, us_per_query=100.0, mem_budget=int(one * 1.6), max_batches=4,
                      max_batch_queries=256) as srv:
        first = srv.submit(0, q(200, 1), 16)       # 20 ms on the device, most of the memory
        deadline = time.time() + 5
        while srv.stats()["batches"] < 1 and time.time() < deadline:
            time.sleep(0.0005)
        big = srv.submit(1, q(200, 2), 16)         # does not fit next to the first
        small = srv.submit(1, q(4, 3), 16)         # fits: goes ahead of `big`
        res = wait_all(srv, [first, big, small])
        assert int(res[small][1][0, 0]) < int(res[big][1][0, 0])
        assert srv.stats()["peak_mem_in_flight"] <= int(one * 1.6)


def test_memory_budget_bounds_batches_in_flight(K):
    # one request's memory is a bit over a third of the budget: at most two in flight
    probe = K.Server.dry(1, m=2000, d=D, us_per_query=0.0, mem_budget=1 << 40)
    probe.wait(probe.submit(0, q(256), 16))
    one = probe.stats()["peak_mem_in_flight"]
    probe.close()
    budget = int(one * 2.5)
    with K.Server.dry(4, m=2000, d=D, us_per_query=40.0, mem_budget=budget, max_batches=8,
                      max_batch_queries=256) as srv:
        subs = [srv.submit(i % 4, q(256, i), 16) for i in range(24)]
        wait_all(srv, subs)
        st = srv.stats()
        assert st["peak_mem_in_flight"] <= budget
        assert st["peak_batches_in_flight"] == 2
        assert st["completed"] == 24


def test_streams_bound_batches_in_flight(K):
    with K.Server.dry(8, m=200, d=D, us_per_query=300.0, max_batches=3) as srv:
        subs = [srv.submit(i % 8, q(4, i), 2) for i in range(16)]
        wait_all(srv, subs)
        assert srv.stats()["peak_batches_in_flight"] == 3


def test_back_pressure(K):
    with K.Server.dry(2, m=200, d=D, us_per_query=20000.0, max_batches=1, max_queue=2) as srv:
        t0 = srv.submit(0, q(10), 2)  # 200 ms on the only stream
        deadline = time.time() + 5
        while srv.stats()["batches"] < 1 and time.time() < deadline:
            time.sleep(0.001)
        t1 = srv.submit(1, q(1), 2)
        t2 = srv.submit(1, q(1), 2)
        with pytest.raises(K.KnnError) as ei:
            srv.submit(0, q(1), 2)
        assert ei.value.status == -5
        assert srv.stats()["rejected_busy"] == 1
        wait_all(srv, [t0, t1, t2])
        srv.wait(srv.submit(0, q(1), 2))  # accepted again once the queue drained


def test_request_over_budget_is_unsupported(K):
    with K.Server.dry(1, m=5000, d=64, us_per_query=0.0, mem_budget=1 << 16) as srv:
        with pytest.raises(K.KnnError) as ei:
            srv.submit(0, np.zeros((512, 64), np.float32), 32)
        assert ei.value.status == -2


def test_submit_validation(K):
    with K.Server.dry(2, m=100, d=D, us_per_query=0.0, max_batch_queries=64) as srv:
        for args in [(2, q(1), 1), (-1, q(1), 1), (0, q(1), 0), (0, q(1), 101)]:
            with pytest.raises(K.KnnError):
                srv.submit(*args)
        with pytest.raises(K.KnnError):
            srv.submit(0, q(65), 1)  # more queries than one batch may hold
        with pytest.raises(ValueError):
            srv.submit(0, np.zeros((3, D + 1), np.float32), 1)


def test_tickets_retire_and_poll(K):
    with K.Server.dry(1, m=100, d=D, us_per_query=5.0) as srv:
        t = srv.submit(0, q(3), 2)
        while (r := srv.poll(t)) is None:
            time.sleep(0.0005)
        dist, idx, lat = r
        assert dist.shape == (3, 2) and lat > 0
        with pytest.raises(K.KnnError):
            srv.poll(t)


def test_destroy_drains_queue(K):
    srv = K.Server.dry(2, m=100, d=D, us_per_query=100.0, max_batches=1, max_batch_queries=4)
    for i in range(10):
        srv.submit(i % 2, q(4, i), 2)
    srv.close()  # returns after every queued request ran


def test_create_validation(K):
    import ctypes

    import paper_0804_1448_amd._lib as L

    lib = L.load()
    h = ctypes.c_void_p()
    good = dict(mem_budget=1 << 20, max_batches=1, max_queue=1, max_batch_queries=1, precision=0, s_extra=-1,
                flags=1, dry_m=10, dry_d=4, dry_us_per_query=0.0)
    for bad in [dict(mem_budget=0), dict(max_batches=0), dict(max_queue=0), dict(max_batch_queries=0),
                dict(precision=7), dict(dry_m=0), dict(dry_d=0)]:
        cfg = L.ServerConfig(**{**good, **bad})
        assert lib.knn_server_create(None, 1, ctypes.byref(cfg), ctypes.byref(h)) == -1, bad
    cfg = L.ServerConfig(**{**good, "flags": 0})
    assert lib.knn_server_create(None, 1, ctypes.byref(cfg), ctypes.byref(h)) == -1  # real server needs sets
    assert lib.knn_server_create(None, 0, ctypes.byref(L.ServerConfig(**good)), ctypes.byref(h)) == -1
    assert lib.knn_server_submit(None, 0, None, 1, 1, None, None, None) == -1
    assert lib.knn_server_destroy(None) == -1
    assert not h.value


def test_cancel_withdraws_waiting_requests_only(K):
    """A waiting request can be withdrawn: it completes at once as
    CANCELLED, its host arrays untouched, and never reaches a batch.  A
    request on the device (or complete) cannot: cancel says so and it
    completes normally."""
    with K.Server.dry(1, m=500, d=D, us_per_query=2000.0, max_batches=1, max_batch_queries=8) as srv:
        first = srv.submit(0, q(8), 3)            # fills the only stream for 16 ms
        time.sleep(0.005)
        later = [srv.submit(0, q(8, i), 3) for i in range(1, 4)]  # each a batch of its own, waiting
        _, dist_w, idx_w = srv._live[later[1]]
        dist_w[:] = -5.0
        idx_w[:] = -9
        assert srv.cancel(later[1]) is True
        with pytest.raises(K.KnnError) as ei:
            srv.wait(later[1])
        assert ei.value.status == -6
        assert np.all(dist_w == -5.0) and np.all(idx_w == -9), "a cancelled request's arrays were written"
        assert srv.cancel(first) is False         # on the device
        d0, i0, _ = srv.wait(first)
        assert np.all(d0 == 0)
        seqs = [srv.wait(t)[1][0, 0] for t in (later[0], later[2])]
        assert seqs == [1, 2], "the cancelled request took a launch"
        with pytest.raises(K.KnnError):
            srv.cancel(first)                     # retired ticket
        st = srv.stats()
        assert st["cancelled"] == 1 and st["batches"] == 3
        assert st["submitted"] == st["completed"] == 4
