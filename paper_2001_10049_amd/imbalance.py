"""Tail imbalance of the extension kernels, from per-wave busy intervals.

The paper measures the alignment stage's load imbalance as the largest
processor's stage time over the average one (section 9, Fig. 8), and notes
that uneven read lengths and early X-drop exits make it impossible to balance
statically.  On one GPU the processors are the compute units: this tool runs
one batch of a workload in the plain form (extensions in task order) and the
batched form (length-binned queue, longest first) with the instrumented
library (libxdrop_stamps.so, every wave of the extension kernels records its
start, end and hardware slot) and reports, per kernel:

  span       first wave start to last wave end
  cu_max_avg largest compute unit's busy time (union of its waves'
             intervals) over the average one: the paper's max/avg
  drain      time from when the kernel's work ran out (the last wave start of
             a one-wave-per-item grid; the first wave end of a persistent
             grid, whose waves leave only when no work is left) to its end,
             as a share of the span
  occ        busy wave-time over (peak resident waves x span)
  partial    share of the span with fewer than half the peak waves resident

    XDROP_LIB=stamps python -m paper_2001_10049_amd.imbalance --workload c3 c4
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

TAGS = {0x01: "k_ext_first<1,16>", 0x20: "k_pair_tier<4>", 0x21: "k_pair2_tier<4>",
        0x22: "k_pair4_tier<4>", 0x80: "k_ext_band"}
for _c in (1, 2, 4, 8, 16):
    TAGS[0x40 + _c] = "k_ext_tier<%d,...>" % _c
PERSISTENT_TAGS = {t for t in TAGS if t != 0x01}
CLOCK_HZ = 100e6  # steady counter


def decode(rec: np.ndarray):
    """rec: (n, 3) uint64 -> dict of arrays (times in us)."""
    t0 = rec[:, 0].astype(np.float64)
    t1 = rec[:, 1].astype(np.float64)
    w = rec[:, 2]
    tag = (w >> np.uint64(56)).astype(np.int64)
    xcc = ((w >> np.uint64(48)) & np.uint64(15)).astype(np.int64)
    hw = ((w >> np.uint64(32)) & np.uint64(0xFFFF)).astype(np.int64)
    items = (w & np.uint64(0xFFFFFFFF)).astype(np.int64)
    # HW_ID: SIMD in bits 4-5, CU 8-11, shader array 12, shader engine 13-15
    cu = (xcc << 8) | (hw >> 8)
    return dict(t0=t0 * 1e6 / CLOCK_HZ, t1=t1 * 1e6 / CLOCK_HZ, tag=tag, cu=cu, items=items)


def union_length(s: np.ndarray, e: np.ndarray) -> float:
    """Total length of the union of intervals [s, e)."""
    o = np.argsort(s, kind="stable")
    s, e = s[o], e[o]
    reach = np.maximum.accumulate(e)
    # a new component starts where s exceeds every earlier end
    gap = np.maximum(s[1:] - reach[:-1], 0.0)
    return float(reach[-1] - s[0] - gap.sum())


def kernel_stats(d: dict, tag: int) -> dict:
    m = d["tag"] == tag
    s, e, cu, items = d["t0"][m], d["t1"][m], d["cu"][m], d["items"][m]
    if s.size == 0:
        return {}
    t_beg, t_end = float(s.min()), float(e.max())
    span = max(t_end - t_beg, 1e-9)
    busy = []
    for c in np.unique(cu):
        k = cu == c
        busy.append(union_length(s[k], e[k]))
    busy = np.asarray(busy)
    # resident waves over time
    ev_t = np.concatenate([s, e])
    ev_d = np.concatenate([np.ones_like(s), -np.ones_like(e)])
    o = np.lexsort((ev_d, ev_t))  # ends before starts at equal times
    ev_t, ev_d = ev_t[o], ev_d[o]
    active = np.cumsum(ev_d)
    dt = np.diff(ev_t, append=t_end)
    peak = float(active.max())
    partial = float(dt[active < 0.5 * peak].sum()) / span
    occ = float((e - s).sum()) / (peak * span)
    if tag in PERSISTENT_TAGS:
        worked = items > 0
        t_dry = float(e[worked].min()) if worked.any() else t_beg
    else:
        t_dry = float(s.max())
    return {"kernel": TAGS.get(tag, hex(tag)), "waves": int(s.size), "items": int(items.sum()),
            "cus": int(busy.size), "span_ms": round(span / 1e3, 3),
            "cu_busy_avg_ms": round(float(busy.mean()) / 1e3, 3),
            "cu_busy_max_ms": round(float(busy.max()) / 1e3, 3),
            "cu_max_avg": round(float(busy.max() / busy.mean()), 3),
            "drain_share": round((t_end - t_dry) / span, 4),
            "occ": round(occ, 4), "partial_share": round(partial, 4),
            "peak_waves": int(peak)}


def run_form(xd, torch, store, pairs, seeds, x, k, form, tuning, cap):
    buf = torch.zeros(cap * 3, dtype=torch.int64, device=pairs.device)
    lib = xd._lib.load()
    # warm up (first-touch of the store, code objects) with recording off
    xd._lib.check(lib.xd_debug_stamps_arm(None, 0))
    kw = dict(x=x, k=k)
    if form == "persistent":
        kw.update(persistent=True, tuning=tuning)
    xd.align_batch(store, pairs, seeds, **kw)
    torch.cuda.synchronize()
    xd._lib.check(lib.xd_debug_stamps_arm(xd._p(buf), cap))
    t = time.perf_counter()
    out = xd.align_batch(store, pairs, seeds, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    import ctypes
    n = ctypes.c_uint32(0)
    xd._lib.check(lib.xd_debug_stamps_count(ctypes.byref(n)))
    xd._lib.check(lib.xd_debug_stamps_arm(None, 0))
    if n.value > cap:
        raise RuntimeError("%d wave records, capacity %d" % (n.value, cap))
    rec = buf[: 3 * n.value].view(-1, 3).cpu().numpy().view(np.uint64)
    d = decode(rec)
    res = {"form": form, "wall_ms": round(wall * 1e3, 3),
           "cells": int(out["cells"].sum())}
    res["kernels"] = [kernel_stats(d, int(tg)) for tg in sorted(np.unique(d["tag"]))]
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", nargs="+", default=["c3", "c4"])
    ap.add_argument("--forms", default="plain,persistent")
    ap.add_argument("--tasks", type=int, default=0,
                    help="use the first N tasks of each workload (0: all)")
    ap.add_argument("--json", default="", help="also append the records to this file")
    args = ap.parse_args(argv)

    import torch
    import synth
    import paper_2001_10049_amd as xd
    if not xd._lib.LIB_PATH.endswith("libxdrop_stamps.so"):
        sys.exit("run with XDROP_LIB=stamps (the instrumented build)")
    lib = xd._lib.load()
    import ctypes
    lib.xd_debug_stamps_arm.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    lib.xd_debug_stamps_arm.restype = ctypes.c_int
    lib.xd_debug_stamps_count.argtypes = [ctypes.POINTER(ctypes.c_uint32)]
    lib.xd_debug_stamps_count.restype = ctypes.c_int
    if not torch.cuda.is_available():
        sys.exit("needs a GPU")
    dev = torch.device("cuda:0")
    from paper_2001_10049_amd import tune
    for name in args.workload:
        print("generating", name, flush=True)
        w = synth.config(name)
        if args.tasks:
            w = w.subset(np.arange(min(args.tasks, w.n_tasks)))
        store = xd.ReadStore.from_workload(w)
        pairs, seeds, x = xd.workload_tensors(w, dev)
        tuning = tune.cached(w) or {}
        # one record per wave: at most one per extension, plus the resident waves
        cap = 2 * int(pairs.shape[0]) + (1 << 20)
        for form in args.forms.split(","):
            res = run_form(xd, torch, store, pairs, seeds, x, w.k, form, tuning, cap)
            res["workload"] = name
            res["tasks"] = int(pairs.shape[0])
            print(json.dumps(res), flush=True)
            if args.json:
                with open(args.json, "a") as f:
                    f.write(json.dumps(res) + "\n")
        store.close()
        del pairs, seeds, x
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
