"""Autotuner for the batched form's tunables (xd_tuning).

Times candidate settings of waves per CU, antidiagonal group length and the X
limits of the 64- and 128-cell first windows on a seeded calibration slice of
a workload, and keeps the fastest.  Results never depend on the tuning, only
speed does.  The winners are cached in tuned.json next to this file, keyed
by device name and a workload signature (set of X values and the median read
length in kbp).

    python -m paper_2001_10049_amd.tune --workload c2 c3     (on a GPU)
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")

SPACE = {
    "waves_per_cu": (16, 24, 28, 32),
    "group_steps": (8, 16),
    "x_tier1": (24, 32, 40),
    "x_tier2": (64, 80, 112),
}


def signature(w) -> str:
    xs = "-".join(str(v) for v in sorted(set(int(v) for v in np.unique(w.x))))
    med = int(np.median(w.length)) // 1000
    return "x%s_L%dk" % (xs, med)


def _device_name() -> str:
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.get_device_name(0)
    except Exception:
        pass
    return "unknown"


def _load_cache() -> dict:
    try:
        return json.load(open(CACHE))
    except (OSError, ValueError):
        return {}


def cached(w, device: str | None = None):
    """Tuning chosen for this workload shape on this device, or None."""
    dev = device or _device_name()
    return _load_cache().get(dev, {}).get(signature(w))


def candidates(w):
    xs = set(int(v) for v in np.unique(w.x))
    keys = list(SPACE)
    for vals in itertools.product(*(SPACE[k] for k in keys)):
        t = dict(zip(keys, vals))
        if t["x_tier2"] < t["x_tier1"]:
            continue
        # the X limits only matter for X values the workload has
        if max(xs) <= min(SPACE["x_tier1"]) and (t["x_tier1"], t["x_tier2"]) != (32, 80):
            continue
        yield t


def time_tuning(store, pairs, seeds, x, k, tuning, reps=3):
    import torch
    import paper_2001_10049_amd as xd
    out = xd._alloc_out(int(pairs.shape[0]), pairs.device, True)
    xd.align_batch(store, pairs, seeds, x=x, k=k, out=out, persistent=True, tuning=tuning)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        xd.align_batch(store, pairs, seeds, x=x, k=k, out=out, persistent=True, tuning=tuning)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def autotune(w, slice_tasks=100000, seed=0, log=print):
    """Sweeps the tuning space on a slice of w; returns (best, table)."""
    import paper_2001_10049_amd as xd
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(w.n_tasks, min(slice_tasks, w.n_tasks), replace=False))
    sub = w.subset(idx)
    store = xd.ReadStore.from_workload(sub)
    pairs, seeds, x = xd.workload_tensors(sub, "cuda")
    table = []
    for t in candidates(sub):
        ms = time_tuning(store, pairs, seeds, x, sub.k, t)
        table.append((ms, t))
        log("%8.3f ms  %s" % (ms, t))
    store.close()
    table.sort(key=lambda r: r[0])
    return table[0][1], table


def main():
    ap = argparse.ArgumentParser(description="autotune the batched form")
    ap.add_argument("--workload", nargs="+", default=["c2", "c3"])
    ap.add_argument("--slice", type=int, default=100000)
    ap.add_argument("--out", default=CACHE, help="where to write the merged cache")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    cache = _load_cache()
    dev = _device_name()
    for name in args.workload:
        w = synth.config(name)
        t0 = time.time()
        best, table = autotune(w, args.slice, log=lambda s: print(name, s, flush=True))
        entry = dict(best)
        cache.setdefault(dev, {})[signature(w)] = entry
        print("%s %s -> %s (%.0f s)" % (name, signature(w), entry, time.time() - t0), flush=True)
    tmp = args.out + ".tmp"
    json.dump(cache, open(tmp, "w"), indent=1, sort_keys=True)
    os.replace(tmp, args.out)


if __name__ == "__main__":
    main()
