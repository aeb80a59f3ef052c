"""xd_align_batch_noalloc (the entry point that allocates nothing) against
xd_align_batch through the C ABI: several calls in a row on one device, each
later one smaller than the first, element by element and bit-exact; and the
size limit of its fixed scratch."""
import ctypes

import numpy as np
import pytest

import synth
from helpers import mutate_codes, rand_codes, workload_from

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402
from paper_2001_10049_amd import _lib  # noqa: E402

KEYS = ("score", "beg", "end", "status", "cells")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def run(entry, store, w, idx=None):
    """Calls `entry` (a C function taking xd_align_batch's arguments) on the
    workload's tasks (or the subset idx); returns host arrays."""
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    if idx is not None:
        sel = torch.from_numpy(np.asarray(idx, np.int64)).cuda()
        pairs, seeds, x = pairs[sel].contiguous(), seeds[sel].contiguous(), x[sel].contiguous()
    n = int(pairs.shape[0])
    out = {"score": torch.full((n,), 7, dtype=torch.int32, device="cuda"),
           "beg": torch.full((n, 2), 7, dtype=torch.int32, device="cuda"),
           "end": torch.full((n, 2), 7, dtype=torch.int32, device="cuda"),
           "status": torch.full((n,), 7, dtype=torch.int32, device="cuda"),
           "cells": torch.full((n,), 7, dtype=torch.int64, device="cuda")}
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = entry(store.handle, _ptr(pairs), _ptr(seeds), _ptr(x), 0, n, w.k, 1, -1, -1,
               _ptr(out["score"]), _ptr(out["beg"]), _ptr(out["end"]), _ptr(out["status"]),
               _ptr(out["cells"]), stream)
    assert rc == _lib.XD_OK, _lib.load().xd_last_error()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def edge_workload():
    rng = np.random.default_rng(5)
    A = rand_codes(rng, 3000)
    B = mutate_codes(rng, A, 0.15)
    K = rand_codes(rng, 17)
    reads = [A, A.copy(), B, K, K.copy(), rand_codes(rng, 2500)]
    tasks = [(0, 1, 1000, 1000, X) for X in (0, 7, 25, 200, 1200)]
    tasks += [(0, 1, 0, 0, 25), (0, 1, 2983, 2983, 25), (3, 4, 0, 0, 25), (0, 5, 100, 100, 25)]
    tasks += [(0, 9, 0, 0, 25), (0, 1, 2990, 0, 25), (0, 1, 5, 5, -1)]  # invalid
    return workload_from(reads, tasks)


def test_noalloc_matches_plain_on_calls_in_a_row():
    lib = _lib.load()
    cases = [("c2", None), ("c3-small", None), ("edge", None), ("c2-small", np.arange(0, 300, 3))]
    sizes = []
    for name, idx in cases:
        w = edge_workload() if name == "edge" else synth.config(name)
        store = xd.ReadStore.from_workload(w)
        try:
            got = run(lib.xd_align_batch_noalloc, store, w, idx)
            ref = run(lib.xd_align_batch, store, w, idx)
            # a second no-alloc call after the plain one: same results again
            again = run(lib.xd_align_batch_noalloc, store, w, idx)
        finally:
            store.close()
        n = got["score"].shape[0]
        sizes.append(n)
        print("noalloc %s: %d tasks" % (name, n), flush=True)
        for key in KEYS:
            bad = np.nonzero((got[key] != ref[key]).reshape(n, -1).any(1))[0]
            assert bad.size == 0, "%s %s differs at %s" % (name, key, bad[:5])
            assert np.array_equal(again[key], ref[key]), (name, key)
        if name == "edge":
            assert (ref["status"] != 0).sum() == 3
    assert sizes[0] > max(sizes[1:]), "later calls must be smaller than the first"


def test_noalloc_rejects_batches_beyond_its_scratch():
    lib = _lib.load()
    w = synth.config("c2-small")
    store = xd.ReadStore.from_workload(w)
    try:
        one = _lib.Tuning(0, 0, 0, 0, 0, 1)
        limit = 64 << 20
        n_fit = 1
        while lib.xd_batch_scratch_bytes(store.handle, 2 * n_fit, ctypes.byref(one)) <= limit:
            n_fit *= 2
        n_big = 4 * n_fit  # at least twice the scratch the fixed area holds
        assert lib.xd_batch_scratch_bytes(store.handle, n_big, ctypes.byref(one)) > 2 * limit
        # real task arrays of that size, so that no pointer is short; the call
        # must refuse before enqueuing anything
        z = torch.zeros((n_big, 2), dtype=torch.int32, device="cuda")
        o = torch.empty((n_big, 2), dtype=torch.int32, device="cuda")
        c = torch.empty(n_big, dtype=torch.int64, device="cuda")
        rc = lib.xd_align_batch_noalloc(store.handle, _ptr(z), _ptr(z), None, 25, n_big, w.k, 1,
                                        -1, -1, _ptr(o), _ptr(o), _ptr(o), _ptr(o), _ptr(c),
                                        None)
        assert rc == _lib.XD_EINVAL
        assert b"scratch" in lib.xd_last_error()
        torch.cuda.synchronize()
    finally:
        store.close()
