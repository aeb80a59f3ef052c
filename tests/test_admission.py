"""Server admission policy on the CPU: HBM budget, slots, batch packing,
FIFO order, cancellation (host logic only; the GPU tests cover the server)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("adm")
    so = str(d / "libadm.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared",
                           "-I" + os.path.join(ROOT, "paper_2001_10049_amd", "csrc"),
                           "-o", so, os.path.join(ROOT, "tests", "admission_shim.cpp")])
    L = ctypes.CDLL(so)
    u64, vp = ctypes.c_uint64, ctypes.c_void_p
    L.adm_new.restype = vp
    L.adm_new.argtypes = [u64, ctypes.c_int, u64, u64]
    L.adm_free.argtypes = [vp]
    L.adm_push.argtypes = [vp, u64, u64, u64]
    L.adm_cancel.argtypes = [vp, u64]
    L.adm_next.argtypes = [vp, ctypes.POINTER(u64), ctypes.c_int]
    L.adm_release.argtypes = [vp, u64]
    L.adm_inflight.argtypes = [vp]
    L.adm_inflight.restype = u64
    L.adm_pending.argtypes = [vp]
    L.adm_pending.restype = u64
    return L


def nxt(L, q):
    buf = (ctypes.c_uint64 * 64)()
    k = L.adm_next(q, buf, 64)
    return [buf[i] for i in range(k)]


def test_budget_forces_queueing_and_packs_batches(lib):
    q = lib.adm_new(1000, 4, 10**9, 100)
    for i in range(1, 6):
        assert lib.adm_push(q, i, 10, 300) == 0
    # 3 x 300 fit in 1000, the fourth waits for memory
    assert nxt(lib, q) == [1, 2, 3]
    assert lib.adm_inflight(q) == 900
    assert nxt(lib, q) == []           # head does not fit the remaining 100
    lib.adm_release(q, 900)
    assert nxt(lib, q) == [4, 5]
    lib.adm_free(q)


def test_slots_limit_batches(lib):
    q = lib.adm_new(10**9, 2, 1, 100)  # one task per batch
    for i in range(1, 5):
        lib.adm_push(q, i, 1, 10)
    assert nxt(lib, q) == [1]
    assert nxt(lib, q) == [2]
    assert nxt(lib, q) == []           # both slots busy
    lib.adm_release(q, 10)
    assert nxt(lib, q) == [3]
    lib.adm_free(q)


def test_fifo_no_overtaking(lib):
    q = lib.adm_new(1000, 8, 10**9, 100)
    lib.adm_push(q, 1, 1, 600)
    assert nxt(lib, q) == [1]
    lib.adm_push(q, 2, 1, 600)         # does not fit now
    lib.adm_push(q, 3, 1, 100)         # would fit, but may not overtake 2
    assert nxt(lib, q) == []
    lib.adm_release(q, 600)
    assert nxt(lib, q) == [2, 3]
    lib.adm_free(q)


def test_over_budget_and_queue_full(lib):
    q = lib.adm_new(1000, 2, 10**9, 2)
    assert lib.adm_push(q, 1, 1, 1001) == -1
    assert lib.adm_push(q, 2, 1, 10) == 0
    assert lib.adm_push(q, 3, 1, 10) == 0
    assert lib.adm_push(q, 4, 1, 10) == -2
    lib.adm_free(q)


def test_cancel_waiting_request(lib):
    q = lib.adm_new(1000, 2, 10**9, 10)
    for i in (1, 2, 3):
        lib.adm_push(q, i, 1, 10)
    assert lib.adm_cancel(q, 2) == 1
    assert lib.adm_cancel(q, 9) == 0
    assert nxt(lib, q) == [1, 3]
    lib.adm_free(q)


def test_batch_task_cap(lib):
    q = lib.adm_new(10**9, 4, 100, 10)
    lib.adm_push(q, 1, 60, 1)
    lib.adm_push(q, 2, 60, 1)
    lib.adm_push(q, 3, 500, 1)         # alone larger than the cap: runs by itself
    assert nxt(lib, q) == [1]
    assert nxt(lib, q) == [2]
    assert nxt(lib, q) == [3]
    lib.adm_free(q)


def test_random_invariants(lib):
    rng = np.random.default_rng(0)
    budget = 5000
    q = lib.adm_new(budget, 3, 10**9, 1000)
    inflight = []
    sizes = {}
    nid = 1
    order = []
    for step in range(2000):
        if rng.random() < 0.6:
            b = int(rng.integers(1, budget + 1))
            sizes[nid] = b
            lib.adm_push(q, nid, 1, b)
            nid += 1
        if inflight and rng.random() < 0.4:
            ids = inflight.pop(0)
            lib.adm_release(q, sum(sizes[i] for i in ids))
        ids = nxt(lib, q)
        if ids:
            inflight.append(ids)
            order += ids
        assert lib.adm_inflight(q) <= budget
        assert len(inflight) <= 3
    assert order == sorted(order)      # admitted in submission order
    lib.adm_free(q)
