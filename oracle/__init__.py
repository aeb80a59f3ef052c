"""Reference X-drop seed-and-extend: TEST INFRASTRUCTURE ONLY.

Plain CPU implementation (xdrop_oracle.c, loaded through ctypes) plus tiny
brute-force checks (brute.py).  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
(`paper_2001_10049_amd`) never does, and the two share no code.

Pins (tests/test_oracle_*.py): exhaustive enumeration of alignments per the
section 2 definition, the textbook full dynamic programme for X = infinity,
hand-worked vectors (tests/golden/), closed forms for identical and contained
reads, and invariants (symmetry, best_X <= best_inf, best >= 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "xdrop_oracle.c")
_SRC_BANDED = os.path.join(_HERE, "banded_oracle.c")
_HDR = os.path.join(_HERE, "xdrop_oracle.h")

TASK_OK, TASK_BAD_READ, TASK_BAD_SEED, TASK_BAD_X = 0, 1, 2, 3
X_MAX = 1 << 20
X_INF = 1 << 40  # no pruning


def build_lib(force: bool = False) -> str:
    """Compile the oracle (plain C, gcc) next to its source."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_BANDED), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC, _SRC_BANDED])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Ext(ctypes.Structure):
    _fields_ = [("best", ctypes.c_int64), ("i", ctypes.c_int64), ("j", ctypes.c_int64),
                ("cells", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("antidiagonals", ctypes.c_int64), ("width_sum", ctypes.c_int64),
                ("width_max", ctypes.c_int64)]


class _Task(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("beg_a", ctypes.c_uint32),
                ("beg_b", ctypes.c_uint32), ("end_a", ctypes.c_uint32),
                ("end_b", ctypes.c_uint32), ("cells", ctypes.c_uint64),
                ("status", ctypes.c_int32)]


class _Banded(ctypes.Structure):
    _fields_ = [("best", ctypes.c_int64), ("i", ctypes.c_int64), ("j", ctypes.c_int64),
                ("cells", ctypes.c_uint64)]


class _BandedTask(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("end_a", ctypes.c_uint32),
                ("end_b", ctypes.c_uint32), ("cells", ctypes.c_uint64),
                ("status", ctypes.c_int32)]


BAND_MAX = 48

_lib = None


def _load():
    global _lib
    if _lib is None:
        build_lib()  # compiles when missing or older than its sources
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        lib.xo_extend.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.POINTER(_Ext), ctypes.POINTER(_Stats)]
        lib.xo_check_params.argtypes = [ctypes.c_int32] * 4
        lib.xo_align_task.argtypes = [vp, vp, vp, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_Task),
                                      ctypes.POINTER(_Stats), ctypes.POINTER(_Stats)]
        lib.xo_align_batch.argtypes = [vp, vp, vp, ctypes.c_uint32, vp, vp, vp, ctypes.c_int32,
                                       ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp,
                                       ctypes.c_int]
        lib.xo_banded.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.POINTER(_Banded)]
        lib.xo_banded_task.argtypes = [vp, vp, vp, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(_BandedTask)]
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.xo_banded_trace.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(_Banded), i64p, i64p, vp,
                                        ctypes.c_int64, i64p]
        _lib = lib
    return _lib


def _u8(seq) -> np.ndarray:
    if isinstance(seq, str):
        m = {"A": 0, "C": 1, "G": 2, "T": 3}
        return np.array([m[c] for c in seq], np.uint8)
    return np.ascontiguousarray(seq, dtype=np.uint8)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def extend(a, b, X, match=1, mismatch=-1, gap=-1, with_stats=False):
    """One X-drop extension of a against b -> (best, i, j, cells[, stats])."""
    a, b = _u8(a), _u8(b)
    # keep a valid pointer for empty inputs
    pa = a if a.size else np.zeros(1, np.uint8)
    pb = b if b.size else np.zeros(1, np.uint8)
    r, s = _Ext(), _Stats()
    rc = _load().xo_extend(_p(pa), a.size, _p(pb), b.size, match, mismatch, gap, int(X),
                           ctypes.byref(r), ctypes.byref(s))
    if rc:
        raise MemoryError("oracle extension failed")
    out = (int(r.best), int(r.i), int(r.j), int(r.cells))
    if with_stats:
        return out + ({"antidiagonals": s.antidiagonals, "width_sum": s.width_sum,
                       "width_max": s.width_max},)
    return out


def check_params(k, match, mismatch, gap) -> bool:
    return _load().xo_check_params(k, match, mismatch, gap) == 0


def align_task(codes, off, length, ra, rb, pa, pb, X, k=17, match=1, mismatch=-1, gap=-1,
               with_stats=False):
    """One seed-and-extend task -> dict(score, beg, end, cells, status)."""
    codes = np.ascontiguousarray(codes, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    length = np.ascontiguousarray(length, np.uint32)
    t, ls, rs = _Task(), _Stats(), _Stats()
    rc = _load().xo_align_task(_p(codes), _p(off), _p(length), length.size, ra, rb, pa, pb,
                               int(X), k, match, mismatch, gap, ctypes.byref(t),
                               ctypes.byref(ls), ctypes.byref(rs))
    if rc:
        raise MemoryError("oracle task failed")
    out = dict(score=t.score, beg=(t.beg_a, t.beg_b), end=(t.end_a, t.end_b), cells=t.cells,
               status=t.status)
    if with_stats:
        out["left_stats"] = {"antidiagonals": ls.antidiagonals, "width_sum": ls.width_sum,
                             "width_max": ls.width_max}
        out["right_stats"] = {"antidiagonals": rs.antidiagonals, "width_sum": rs.width_sum,
                              "width_max": rs.width_max}
    return out


def align_batch(codes, off, length, pairs, seeds, x=None, x_scalar=0, k=17, match=1,
                mismatch=-1, gap=-1, n_threads=None):
    """n tasks -> (dict of arrays, threads used).

    pairs, seeds: uint32[n, 2]; x: int32[n] or None (x_scalar for all).
    """
    codes = np.ascontiguousarray(codes, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    length = np.ascontiguousarray(length, np.uint32)
    pairs = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
    seeds = np.ascontiguousarray(seeds, np.uint32).reshape(-1, 2)
    n = pairs.shape[0]
    xs = None if x is None else np.ascontiguousarray(x, np.int32)
    score = np.zeros(n, np.int32)
    beg = np.zeros((n, 2), np.uint32)
    end = np.zeros((n, 2), np.uint32)
    status = np.zeros(n, np.int32)
    cells = np.zeros(n, np.uint64)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    dummy = np.zeros(1, np.uint32)
    used = _load().xo_align_batch(
        _p(codes), _p(off), _p(length), length.size, _p(pairs if n else dummy),
        _p(seeds if n else dummy), None if xs is None else _p(xs), int(x_scalar), n, k, match,
        mismatch, gap, _p(score if n else dummy), _p(beg if n else dummy),
        _p(end if n else dummy), _p(status if n else dummy), _p(cells if n else dummy),
        int(n_threads))
    if used < 0:
        raise ValueError("oracle rejected the batch parameters (or ran out of memory)")
    return dict(score=score, beg=beg, end=end, status=status, cells=cells), used


def align_workload(w, x=None, n_threads=None, **kw):
    """Oracle results for every task of a synth.Workload."""
    pairs = np.stack([w.ra, w.rb], 1)
    seeds = np.stack([w.pa, w.pb], 1)
    res, _ = align_batch(w.codes, w.off, w.length, pairs, seeds,
                         x=w.x if x is None else x, k=w.k, n_threads=n_threads, **kw)
    return res


def banded(a, b, c, w, match=1, mismatch=-1, gap=-1):
    """Banded Smith-Waterman (banded_oracle.c) -> (best, i, j, cells)."""
    a, b = _u8(a), _u8(b)
    pa = a if a.size else np.zeros(1, np.uint8)
    pb = b if b.size else np.zeros(1, np.uint8)
    r = _Banded()
    if _load().xo_banded(_p(pa), a.size, _p(pb), b.size, int(c), int(w), match, mismatch, gap,
                         ctypes.byref(r)):
        raise MemoryError("banded oracle failed")
    return int(r.best), int(r.i), int(r.j), int(r.cells)


OP_M, OP_I, OP_D = 0, 1, 2  # run-length entries: length << 2 | op


def banded_trace(a, b, c, w, match=1, mismatch=-1, gap=-1):
    """Banded Smith-Waterman with traceback (banded_oracle.c) -> (best, i, j,
    cells, beg_i, beg_j, ops uint32 array of run-length entries)."""
    a, b = _u8(a), _u8(b)
    pa = a if a.size else np.zeros(1, np.uint8)
    pb = b if b.size else np.zeros(1, np.uint8)
    r = _Banded()
    bi, bj, nops = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    cap = a.size + b.size + 1
    ops = np.zeros(cap, np.uint32)
    if _load().xo_banded_trace(_p(pa), a.size, _p(pb), b.size, int(c), int(w), match, mismatch,
                               gap, ctypes.byref(r), ctypes.byref(bi), ctypes.byref(bj), _p(ops),
                               cap, ctypes.byref(nops)):
        raise MemoryError("banded traceback oracle failed")
    return (int(r.best), int(r.i), int(r.j), int(r.cells), int(bi.value), int(bj.value),
            ops[:nops.value].copy())


def banded_trace_batch(codes, off, length, pairs, seeds, w, k=17, match=1, mismatch=-1, gap=-1):
    """Banded tasks with traceback -> dict(score, beg[n, 2], end[n, 2], cells,
    status, ops = list of run-length arrays); statuses as banded_batch."""
    base = banded_batch(codes, off, length, pairs, seeds, w, k, match, mismatch, gap)
    codes = np.ascontiguousarray(codes, np.uint8)
    pairs = np.asarray(pairs, np.uint32).reshape(-1, 2)
    seeds = np.asarray(seeds, np.uint32).reshape(-1, 2)
    n = pairs.shape[0]
    ws = np.broadcast_to(np.asarray(w, np.int64), (n,))
    base["beg"] = np.zeros((n, 2), np.uint32)
    base["ops"] = []
    for t in range(n):
        if base["status"][t] != 0:
            base["ops"].append(np.zeros(0, np.uint32))
            continue
        ra, rb = int(pairs[t, 0]), int(pairs[t, 1])
        A = codes[int(off[ra]):int(off[ra]) + int(length[ra])]
        B = codes[int(off[rb]):int(off[rb]) + int(length[rb])]
        best, i, j, cells, bi, bj, ops = banded_trace(A, B, int(seeds[t, 0]) - int(seeds[t, 1]),
                                                      int(ws[t]), match, mismatch, gap)
        assert (best, i, j, cells) == (base["score"][t], base["end"][t][0], base["end"][t][1],
                                       base["cells"][t])
        base["beg"][t] = (bi, bj)
        base["ops"].append(ops)
    return base


def banded_batch(codes, off, length, pairs, seeds, w, k=17, match=1, mismatch=-1, gap=-1):
    """Banded tasks (band around each seed's diagonal) -> dict(score, end[n, 2],
    cells, status); w: one half-width or one per task."""
    codes = np.ascontiguousarray(codes, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    length = np.ascontiguousarray(length, np.uint32)
    pairs = np.asarray(pairs, np.uint32).reshape(-1, 2)
    seeds = np.asarray(seeds, np.uint32).reshape(-1, 2)
    n = pairs.shape[0]
    ws = np.broadcast_to(np.asarray(w, np.int64), (n,))
    out = dict(score=np.zeros(n, np.int32), end=np.zeros((n, 2), np.uint32),
               cells=np.zeros(n, np.uint64), status=np.zeros(n, np.int32))
    lib = _load()
    r = _BandedTask()
    for t in range(n):
        if lib.xo_banded_task(_p(codes), _p(off), _p(length), length.size, int(pairs[t, 0]),
                              int(pairs[t, 1]), int(seeds[t, 0]), int(seeds[t, 1]), int(ws[t]),
                              k, match, mismatch, gap, ctypes.byref(r)):
            raise ValueError("banded oracle rejected the task parameters")
        out["score"][t] = r.score
        out["end"][t] = (r.end_a, r.end_b)
        out["cells"][t] = r.cells
        out["status"][t] = r.status
    return out
