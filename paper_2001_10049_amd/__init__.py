"""X-drop seed-and-extend alignment of long-read pairs on MI355X.

Thin Python binding over libxdrop.so (C ABI in include/xdrop.h).  Every step
of the alignment runs in the library's HIP kernels; this module only moves
arguments: host arrays for the read store, torch device tensors for task
inputs and results, and the caller's HIP stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (BAND_MAX, READ_MAX, SCORE_LIMIT, TASK_BAD_READ, TASK_BAD_SEED,  # noqa
                   TASK_BAD_X, TASK_BAND_OVERFLOW, TASK_NO_SEED, TASK_OK, X_MAX, XdropError,
                   TASK_OPS_OVERFLOW, TASK_TRACE_FAULT, OP_M, OP_I, OP_D)


def _p(a) -> ctypes.c_void_p:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())


def pack_reads(codes, off, length):
    """Host 2-bit packing (library routine) -> (words uint32, word_off uint64)."""
    lib = _lib.load()
    codes = np.ascontiguousarray(codes, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    length = np.ascontiguousarray(length, np.uint32)
    n = ctypes.c_uint64(0)
    _lib.check(lib.xd_pack_reads(_p(codes), _p(off), _p(length), length.size, None, None,
                                 ctypes.byref(n)))
    words = np.zeros(max(int(n.value), 1), np.uint32)
    woff = np.zeros(max(length.size, 1), np.uint64)
    _lib.check(lib.xd_pack_reads(_p(codes), _p(off), _p(length), length.size, _p(words),
                                 _p(woff), ctypes.byref(n)))
    return words[:int(n.value)], woff[:length.size]


class ReadStore:
    """Device-resident 2-bit read store (xd_store)."""

    def __init__(self, codes, off, length):
        lib = _lib.load()
        codes = np.ascontiguousarray(codes, np.uint8)
        off = np.ascontiguousarray(off, np.uint64)
        length = np.ascontiguousarray(length, np.uint32)
        h = ctypes.c_void_p()
        _lib.check(lib.xd_store_create_from_codes(_p(codes), _p(off), _p(length),
                                                  length.size, ctypes.byref(h)))
        self._h = h
        self.n_reads = int(length.size)

    @classmethod
    def from_workload(cls, w):
        return cls(w.codes, w.off, w.length)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("store is closed")
        return self._h

    def info(self):
        b, n, mx = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32()
        _lib.check(_lib.load().xd_store_info(self.handle, ctypes.byref(b), ctypes.byref(n),
                                             ctypes.byref(mx)))
        return dict(device_bytes=b.value, n_reads=n.value, max_len=mx.value)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().xd_store_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(name, t, n_items, dtype_bytes):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if not t.is_contiguous() or t.element_size() != dtype_bytes or t.numel() != n_items:
        raise ValueError("%s: need a contiguous %d-byte tensor with %d elements" %
                         (name, dtype_bytes, n_items))


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, _lib.Tuning):
        return ctypes.byref(t)
    return ctypes.byref(_tuning_struct(t))


def _tuning_struct(t) -> "_lib.Tuning":
    t = t or {}
    return _lib.Tuning(*(int(t.get(f, 0)) for f, _ in _lib.Tuning._fields_))


def _alloc_out(n, dev, with_cells):
    import torch
    return dict(score=torch.empty(n, dtype=torch.int32, device=dev),
                beg=torch.empty((n, 2), dtype=torch.int32, device=dev),
                end=torch.empty((n, 2), dtype=torch.int32, device=dev),
                status=torch.empty(n, dtype=torch.int32, device=dev),
                cells=torch.empty(n, dtype=torch.int64, device=dev) if with_cells else None)


def _check_batch(pairs, seeds, x, out):
    n = int(pairs.shape[0])
    _check_dev("pairs", pairs, 2 * n, 4)
    _check_dev("seeds", seeds, 2 * n, 4)
    if x is not None:
        _check_dev("x", x, n, 4)
    if out is None:
        out = _alloc_out(n, pairs.device, True)
    _check_dev("score", out["score"], n, 4)
    _check_dev("beg", out["beg"], 2 * n, 4)
    _check_dev("end", out["end"], 2 * n, 4)
    _check_dev("status", out["status"], n, 4)
    if out.get("cells") is not None:
        _check_dev("cells", out["cells"], n, 8)
    return n, out


def align_batch(store: ReadStore, pairs, seeds, x=None, x_scalar=0, k=17, match=1,
                mismatch=-1, gap=-1, out=None, stream=None, persistent=False, tuning=None,
                noalloc=False):
    """Aligns n tasks on the GPU (xd_align_batch, or the batched form
    xd_align_batch_persistent when persistent=True, or xd_align_batch_noalloc,
    which takes no memory, when noalloc=True; pass `out` then to allocate
    nothing on the Python side either).

    pairs, seeds: int32/uint32 device tensors [n, 2]; x: int32 [n] or None.
    Returns dict(score int32 [n], beg int32 [n,2], end int32 [n,2],
    status int32 [n], cells int64 [n]) of device tensors (coordinates hold the
    uint32 bit patterns).  Asynchronous on `stream` (default: current).
    tuning: dict(waves_per_cu, group_steps, order, x_tier1, x_tier2,
    band_blocks) for the batched form (see xd_tuning).
    """
    n, out = _check_batch(pairs, seeds, x, out)
    lib = _lib.load()
    args = (store.handle, _p(pairs), _p(seeds), _p(x), int(x_scalar), n, int(k), int(match),
            int(mismatch), int(gap), _p(out["score"]), _p(out["beg"]), _p(out["end"]),
            _p(out["status"]), _p(out.get("cells")))
    if persistent:
        _lib.check(lib.xd_align_batch_persistent(*args, _tuning(tuning), _stream_ptr(stream)))
    elif noalloc:
        _lib.check(lib.xd_align_batch_noalloc(*args, _stream_ptr(stream)))
    else:
        _lib.check(lib.xd_align_batch(*args, _stream_ptr(stream)))
    return out


def banded_batch(store: ReadStore, pairs, seeds, w=None, w_scalar=32, k=17, match=1,
                 mismatch=-1, gap=-1, stream=None):
    """Banded Smith-Waterman (xd_banded_batch) around each seed's diagonal.

    pairs, seeds: [n, 2] 4-byte device tensors; w: int32 [n] or None.  Returns
    dict(score int32 [n], end int32 [n, 2], status int32 [n], cells int64 [n])."""
    import torch
    n = int(pairs.shape[0])
    dev = pairs.device
    _check_dev("pairs", pairs, 2 * n, 4)
    _check_dev("seeds", seeds, 2 * n, 4)
    if w is not None:
        _check_dev("w", w, n, 4)
    out = dict(score=torch.empty(n, dtype=torch.int32, device=dev),
               end=torch.empty((n, 2), dtype=torch.int32, device=dev),
               status=torch.empty(n, dtype=torch.int32, device=dev),
               cells=torch.empty(n, dtype=torch.int64, device=dev))
    lib = _lib.load()
    _lib.check(lib.xd_banded_batch(store.handle, _p(pairs), _p(seeds), _p(w), int(w_scalar), n,
                                   int(k), int(match), int(mismatch), int(gap), _p(out["score"]),
                                   _p(out["end"]), _p(out["status"]), _p(out["cells"]),
                                   _stream_ptr(stream)))
    return out


def banded_traceback(store: ReadStore, pairs, seeds, w=None, w_scalar=32, k=17, match=1,
                     mismatch=-1, gap=-1, max_ops=4096, trace_budget=0, stream=None):
    """Banded Smith-Waterman with the alignment path (xd_banded_traceback).

    Returns banded_batch's dict plus beg int32 [n, 2], ops int32 [n, max_ops]
    (run-length entries run << 2 | op, op OP_M / OP_I / OP_D; the first
    n_ops[t] of row t are valid) and n_ops int32 [n].  Synchronous."""
    import torch
    n = int(pairs.shape[0])
    dev = pairs.device
    _check_dev("pairs", pairs, 2 * n, 4)
    _check_dev("seeds", seeds, 2 * n, 4)
    if w is not None:
        _check_dev("w", w, n, 4)
    out = dict(score=torch.empty(n, dtype=torch.int32, device=dev),
               beg=torch.empty((n, 2), dtype=torch.int32, device=dev),
               end=torch.empty((n, 2), dtype=torch.int32, device=dev),
               status=torch.empty(n, dtype=torch.int32, device=dev),
               cells=torch.empty(n, dtype=torch.int64, device=dev),
               ops=torch.empty((n, max(int(max_ops), 1)), dtype=torch.int32, device=dev),
               n_ops=torch.empty(n, dtype=torch.int32, device=dev))
    lib = _lib.load()
    _lib.check(lib.xd_banded_traceback(
        store.handle, _p(pairs), _p(seeds), _p(w), int(w_scalar), n, int(k), int(match),
        int(mismatch), int(gap), int(max_ops), int(trace_budget), _p(out["score"]),
        _p(out["beg"]), _p(out["end"]), _p(out["status"]), _p(out["cells"]), _p(out["ops"]),
        _p(out["n_ops"]), _stream_ptr(stream)))
    return out


def find_overlaps(store: ReadStore, k=17, m=8, bloom_bits=0, capacity=None, stream=None,
                  table_slots=0, strands=1):
    """Candidate read pairs sharing a retained k-mer (xd_find_overlaps_strands).

    strands: 1 = forward k-mers; 2 = canonical k-mers over both strands,
    with a reverse-strand flag per pair.  capacity: (max_pairs, max_seeds) to
    allocate at once; None asks the library for the counts first (one extra
    run).  bloom_bits and table_slots size the first filter and the first
    hash table (0: the library's choice); they change speed and memory, never
    the result.  Returns dict(pairs int32 [P, 2], rc uint8 [P], seed_off
    int64 [P + 1], seeds int32 [S, 2] device tensors, counts dict) or raises
    XdropError(XD_EAGAIN) when capacity is too small."""
    import torch
    lib = _lib.load()
    cnt = _lib.OverlapCounts()
    st = _stream_ptr(stream)
    if capacity is None:
        _lib.check(lib.xd_find_overlaps_strands(store.handle, int(k), int(m), int(bloom_bits),
                                                int(table_slots), int(strands), 0, None, None,
                                                None, 0, None, ctypes.byref(cnt), st))
        capacity = (cnt.pairs, cnt.seeds)
    max_pairs, max_seeds = int(capacity[0]), int(capacity[1])
    dev = torch.device("cuda", torch.cuda.current_device())
    pairs = torch.empty((max(max_pairs, 1), 2), dtype=torch.int32, device=dev)
    rc = torch.zeros(max(max_pairs, 1), dtype=torch.uint8, device=dev)
    seed_off = torch.empty(max_pairs + 1, dtype=torch.int64, device=dev)
    seeds = torch.empty((max(max_seeds, 1), 2), dtype=torch.int32, device=dev)
    _lib.check(lib.xd_find_overlaps_strands(store.handle, int(k), int(m), int(bloom_bits),
                                            int(table_slots), int(strands), max_pairs,
                                            _p(pairs), _p(rc), _p(seed_off), max_seeds,
                                            _p(seeds), ctypes.byref(cnt), st))
    counts = {f: int(getattr(cnt, f)) for f, _ in _lib.OverlapCounts._fields_}
    P, S = counts["pairs"], counts["seeds"]
    return dict(pairs=pairs[:P], rc=rc[:P], seed_off=seed_off[:P + 1], seeds=seeds[:S],
                counts=counts)


def align_pairs(store: ReadStore, pairs, seed_off, seeds, rc=None, x=None, x_scalar=0,
                min_dist=17, max_seeds=0, k=17, match=1, mismatch=-1, gap=-1, n_seeds=None,
                stream=None, tuning=None):
    """Multi-seed pair alignment (xd_align_pairs): per pair, choose seeds from
    its list, align each, keep the best.

    pairs: [n, 2] 4-byte device tensor; seed_off: int64 [n + 1]; seeds:
    [S, 2] 4-byte; rc: uint8 [n] or None; x: int32 [n] or None.  n_seeds
    defaults to seed_off[-1] (read back from the device).  Returns dict of
    device tensors per pair: score, beg, end, status, seed_idx, n_kept, cells.
    """
    import torch
    n = int(pairs.shape[0])
    dev = pairs.device
    _check_dev("pairs", pairs, 2 * n, 4)
    _check_dev("seed_off", seed_off, n + 1, 8)
    if n_seeds is None:
        n_seeds = int(seed_off[-1].item()) if n else 0
    if n_seeds:
        _check_dev("seeds", seeds, 2 * n_seeds, 4)
    if rc is not None:
        _check_dev("rc", rc, n, 1)
    if x is not None:
        _check_dev("x", x, n, 4)
    out = dict(score=torch.empty(n, dtype=torch.int32, device=dev),
               beg=torch.empty((n, 2), dtype=torch.int32, device=dev),
               end=torch.empty((n, 2), dtype=torch.int32, device=dev),
               status=torch.empty(n, dtype=torch.int32, device=dev),
               seed_idx=torch.empty(n, dtype=torch.int32, device=dev),
               n_kept=torch.empty(n, dtype=torch.int32, device=dev),
               cells=torch.empty(n, dtype=torch.int64, device=dev))
    lib = _lib.load()
    _lib.check(lib.xd_align_pairs(
        store.handle, n, _p(pairs), _p(rc), _p(seed_off), _p(seeds) if n_seeds else None,
        int(n_seeds), _p(x), int(x_scalar), int(min_dist), int(max_seeds), int(k), int(match),
        int(mismatch), int(gap), _p(out["score"]), _p(out["beg"]), _p(out["end"]),
        _p(out["status"]), _p(out["seed_idx"]), _p(out["n_kept"]), _p(out["cells"]),
        _tuning(tuning), _stream_ptr(stream)))
    return out


class Plan:
    """A captured batch (xd_plan): fixed buffers, replayed with launch()."""

    def __init__(self, store, pairs, seeds, x=None, x_scalar=0, k=17, match=1, mismatch=-1,
                 gap=-1, out=None, tuning=None):
        n, out = _check_batch(pairs, seeds, x, out)
        self.out = out
        self._keep = (store, pairs, seeds, x)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().xd_plan_create(
            store.handle, _p(pairs), _p(seeds), _p(x), int(x_scalar), n, int(k), int(match),
            int(mismatch), int(gap), _p(out["score"]), _p(out["beg"]), _p(out["end"]),
            _p(out["status"]), _p(out.get("cells")), _tuning(tuning), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _lib.check(_lib.load().xd_plan_launch(self._h, _stream_ptr(stream)))
        return self.out

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().xd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workload_tensors(w, device="cuda"):
    """Task arrays of a synth.Workload as device tensors (pairs, seeds, x)."""
    import torch
    pairs = torch.from_numpy(np.stack([w.ra, w.rb], 1).astype(np.int32)).to(device)
    seeds = torch.from_numpy(np.stack([w.pa, w.pb], 1).astype(np.int32)).to(device)
    x = torch.from_numpy(w.x.astype(np.int32)).to(device)
    return pairs, seeds, x


def release_memory() -> None:
    """Hands the library's cached scratch memory back to the device
    (xd_release_memory)."""
    _lib.check(_lib.load().xd_release_memory())


def profile_enable(on: bool = True) -> None:
    """Start/stop per-kernel event timing of xd_align_batch calls."""
    _lib.check(_lib.load().xd_profile_enable(1 if on else 0))


def profile_read(reset: bool = True) -> dict:
    """Waits for recorded batches and returns the summed per-stage profile."""
    p = _lib.Profile()
    _lib.check(_lib.load().xd_profile_read(ctypes.byref(p), 1 if reset else 0))
    return {f: getattr(p, f) for f, _ in _lib.Profile._fields_}


def batch_scratch_bytes(n: int, store=None, tuning=None) -> int:
    """Device scratch bytes of one batch call of n tasks (xd_batch_scratch_bytes);
    without a store the band tier's rows are left out."""
    t = _tuning_struct(tuning)
    return int(_lib.load().xd_batch_scratch_bytes(store.handle if store is not None else None,
                                                  int(n), ctypes.byref(t)))


def request_bytes(n: int) -> int:
    """Device bytes a server request of n tasks holds while in flight."""
    return int(_lib.load().xd_server_request_bytes(int(n)))


def server_fixed_bytes(store, slots=0, tuning=None) -> int:
    """Device bytes a server on this store holds whatever its load (each slot's
    band-tier rows); requests share the rest of hbm_budget_bytes."""
    cfg = _lib.ServerConfig(0, int(slots), 0, 0, 17, 1, -1, -1, _tuning_struct(tuning))
    return int(_lib.load().xd_server_fixed_bytes(store.handle, ctypes.byref(cfg)))


class Server:
    """Request server over a resident read store (xd_server).

    submit() copies host task arrays and returns a request id; poll() returns
    None while the request is pending, else its results (host numpy arrays)
    and timing info.
    """

    def __init__(self, store, hbm_budget_bytes=0, slots=0, max_batch_tasks=0, max_pending=0,
                 k=17, match=1, mismatch=-1, gap=-1, tuning=None):
        cfg = _lib.ServerConfig(int(hbm_budget_bytes), int(slots), int(max_batch_tasks),
                                int(max_pending), int(k), int(match), int(mismatch), int(gap),
                                _tuning_struct(tuning))
        h = ctypes.c_void_p()
        _lib.check(_lib.load().xd_server_create(store.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._store = store
        self._n = {}

    def submit(self, pairs, seeds, x=None, x_scalar=0) -> int:
        pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
        seeds = np.ascontiguousarray(seeds, np.uint32).reshape(-1, 2)
        n = pairs.shape[0]
        xs = None if x is None else np.ascontiguousarray(x, np.int32)
        rid = ctypes.c_uint64()
        _lib.check(_lib.load().xd_server_submit(self._h, _p(pairs), _p(seeds), _p(xs),
                                                int(x_scalar), n, ctypes.byref(rid)))
        self._n[rid.value] = n
        return rid.value

    def poll(self, rid: int, timeout_ms: int = 0):
        n = self._n[rid]
        out = dict(score=np.empty(n, np.int32), beg=np.empty((n, 2), np.uint32),
                   end=np.empty((n, 2), np.uint32), status=np.empty(n, np.int32),
                   cells=np.empty(n, np.uint64))
        info = _lib.RequestInfo()
        rc = _lib.load().xd_server_poll(self._h, rid, int(timeout_ms), _p(out["score"]),
                                        _p(out["beg"]), _p(out["end"]), _p(out["status"]),
                                        _p(out["cells"]), ctypes.byref(info))
        if rc == _lib.XD_EAGAIN:
            return None
        del self._n[rid]
        _lib.check(rc)
        out["info"] = {f: getattr(info, f) for f, _ in _lib.RequestInfo._fields_}
        return out

    def cancel(self, rid: int) -> None:
        _lib.check(_lib.load().xd_server_cancel(self._h, rid))
        self._n.pop(rid, None)

    def stats(self) -> dict:
        c = _lib.ServerCounters()
        _lib.check(_lib.load().xd_server_stats(self._h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in _lib.ServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().xd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
