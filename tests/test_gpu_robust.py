"""GPU tests of the library's failure handling and thread discipline.

* A forced allocation failure (the KNN_FAIL_ALLOC test hook) returns
  KNN_ERR_OOM and leaves the outputs and the handle pointer untouched.
* Float16 storage rejects reference values the format cannot hold.
* Two host threads searching on one stream (the library then shares one
  workspace between them, growing it as sizes change) each get the result
  they get alone.
* A handle searched on a side stream is destroyed safely right after the
  search is enqueued (destroy waits for the handle's own work).
"""
from __future__ import annotations

import ctypes
import os
import sys
import threading

import numpy as np
import pytest

import synthdata
from oracle.check import compare

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


def test_injected_allocation_failure_leaves_outputs(K):
    import torch

    banner("injected allocation failure")
    lib = K.load()
    Q = torch.from_numpy(synthdata.uniform((300, 20), 61, 1)).cuda()
    R = torch.from_numpy(synthdata.uniform((2000, 20), 61, 0)).cuda()
    dist = torch.full((300, 5), -3.0, device="cuda")
    idx = torch.full((300, 5), -3, dtype=torch.int32, device="cuda")
    side = torch.cuda.Stream()  # a stream the library has no workspace for yet
    os.environ["KNN_FAIL_ALLOC"] = "1"
    try:
        st = lib.knn_search(ctypes.c_void_p(Q.data_ptr()), 300, ctypes.c_void_p(R.data_ptr()), 2000, 20, 5, 0,
                            ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                            ctypes.c_void_p(side.cuda_stream))
    finally:
        os.environ.pop("KNN_FAIL_ALLOC", None)
    assert st == -3, st
    assert "injected" in lib.knn_last_error().decode()
    torch.cuda.synchronize()
    assert bool((dist == -3.0).all()) and bool((idx == -3).all())
    # the same call succeeds once the hook is spent
    with torch.cuda.stream(side):
        d2, i2 = K.search(Q, R, 5)
    torch.cuda.synchronize()
    assert compare(Q.cpu().numpy(), R.cpu().numpy(), 5, "l2", d2.cpu().numpy(), i2.cpu().numpy())["ok"]

    # a reference set whose third allocation fails: no handle, status OOM
    h = ctypes.c_void_p(0x1234)
    os.environ["KNN_FAIL_ALLOC"] = "3"
    try:
        st = lib.knn_create_refs(ctypes.c_void_p(R.data_ptr()), 2000, 20, 1, 1, None, ctypes.byref(h))
    finally:
        os.environ.pop("KNN_FAIL_ALLOC", None)
    assert st == -3 and not h.value, (st, h.value)


def test_fp16_storage_rejects_out_of_range_rows(K):
    import torch

    banner("fp16 range check")
    R = synthdata.uniform((500, 8), 62, 0)
    R[123, 5] = 7.0e4  # beyond 65504 when stored without translation
    Rd = torch.from_numpy(R).cuda()
    with pytest.raises(K.KnnError) as e:
        K.Refs(Rd, storage="fp16", keep_fp32_master=False)
    assert e.value.status == -2 and "float16" in str(e.value)
    # in range once translated by the set's centre (the first rows' mean):
    # the master path stores x - c, well inside the float16 range here
    R2 = synthdata.uniform((500, 8), 62, 0) + np.float32(6.0e4)
    refs = K.Refs(torch.from_numpy(R2).cuda(), storage="fp16", keep_fp32_master=True)
    refs.close()
    # bfloat16 holds any finite float32 below its own maximum
    refs = K.Refs(torch.from_numpy(R2).cuda(), storage="bf16", keep_fp32_master=False)
    refs.close()


def test_two_threads_one_stream(K):
    import torch

    banner("two threads, one stream")
    cases = []
    for t in range(2):
        for j, (n, m, d, k) in enumerate([(900, 4000, 32, 10), (4000, 12000, 64, 20), (300, 2000, 16, 5)]):
            Q = synthdata.uniform((n, d), 6300 + 10 * t + j, 1)
            R = synthdata.uniform((m, d), 6300 + 10 * t + j, 0)
            cases.append((t, Q, R, k, torch.from_numpy(Q).cuda(), torch.from_numpy(R).cuda()))
    alone = {}
    for t, Q, R, k, Qd, Rd in cases:
        d_, i_ = K.search(Qd, Rd, k)
        alone[id(Q)] = (d_.cpu().numpy(), i_.cpu().numpy())
    stream = torch.cuda.Stream()
    got = {}
    errors = []

    def worker(t):
        try:
            with torch.cuda.stream(stream):
                for rep in range(6):
                    for tt, Q, R, k, Qd, Rd in cases:
                        if tt == t:
                            got[(id(Q), rep)] = K.search(Qd, Rd, k, stream=stream)
        except Exception as e:  # surfaced below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors
    torch.cuda.synchronize()
    for (key, rep), (d_, i_) in got.items():
        ad, ai = alone[key]
        assert np.array_equal(ad, d_.cpu().numpy()) and np.array_equal(ai, i_.cpu().numpy()), (key, rep)


def test_destroy_waits_for_side_stream_search(K):
    import torch

    banner("destroy after side-stream search")
    R = synthdata.uniform((200000, 64), 64, 0)
    Q = synthdata.uniform((4096, 64), 64, 1)
    Rd, Qd = torch.from_numpy(R).cuda(), torch.from_numpy(Q).cuda()
    refs = K.Refs(Rd, storage="fp16", keep_fp32_master=True)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        dist, idx = refs.search(Qd, 16, "l2", precision="fp16", stream=side)
    refs.close()  # must wait for the search above before freeing the rows
    side.synchronize()
    rows = np.arange(0, 4096, 257)
    rep = compare(Q, R, 16, "l2", dist.cpu().numpy(), idx.cpu().numpy(), rows=rows)
    assert rep["bad_index_rows"] == 0 and rep["bad_pair"] == 0 and rep["recall"] >= 0.999, rep
