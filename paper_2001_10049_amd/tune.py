"""Autotuner for the batched form's tunables (xd_tuning).

Times candidate settings on a seeded calibration slice of a workload and
keeps the fastest.  The slice is a 1 % sample of the tasks (at least 2,000),
repeated until the launch holds at least 200,000 tasks: the sample carries
the workload's mix of X values and lengths, the repetition gives the launch
the full workload's scale, so that waves per CU is judged where the machine
is full rather than on a short launch whose tail favours few waves (a
20,000-task slice of c2 picked 16 waves per CU, 11 % slower on c2 itself
than 24).  Per X bin the tuner picks the first window (64, 128 or
256 cells: the X limits x_tier1 and x_tier2), per length bin the queue
order (longest first, or task order), and beside them waves per CU, the
antidiagonal group length and, when the slice sends any extension to the
band tier, the band tier's workgroup count.  Results never depend on the
tuning, only speed does.  The winners are cached in tuned.json next to this
file, keyed by the device's architecture and compute-unit count (for
example gfx950_256cu) and a workload signature (set of X values and the
median read length in kbp).

    python -m paper_2001_10049_amd.tune --workload c2 c3 c4     (on a GPU)
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
    "x_tier1": (24, 32, 40, 56),
    "x_tier2": (64, 80, 112),
    "order": (1, 2),
}
BAND_BLOCKS = (1, 4, 16, 64)
SLICE_FRACTION = 0.01
SAMPLE_MIN = 2000
LAUNCH_MIN = 200000


def signature(w) -> str:
    xs = "-".join(str(v) for v in sorted(set(int(v) for v in np.unique(w.x))))
    med = int(np.median(w.length)) // 1000
    return "x%s_L%dk" % (xs, med)


def device_key() -> str:
    """gfx architecture and compute-unit count of device 0 (the marketing
    name is not reliable: it depends on the host's device-id tables)."""
    try:
        import torch
        if torch.cuda.is_available():
            p = torch.cuda.get_device_properties(0)
            arch = str(getattr(p, "gcnArchName", "unknown")).split(":")[0]
            return "%s_%dcu" % (arch, p.multi_processor_count)
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
    dev = device or device_key()
    return _load_cache().get(dev, {}).get(signature(w))


def candidates(w):
    xs = sorted(set(int(v) for v in np.unique(w.x)))
    keys = list(SPACE)
    seen = set()
    for vals in itertools.product(*(SPACE[k] for k in keys)):
        t = dict(zip(keys, vals))
        if t["x_tier2"] < t["x_tier1"]:
            continue
        # the X limits only matter through the first window each X value of
        # the workload gets: one candidate per distinct assignment
        firsts = tuple(0 if x <= t["x_tier1"] else 1 if x <= t["x_tier2"] else 2 for x in xs)
        key = (t["waves_per_cu"], t["group_steps"], t["order"], firsts)
        if key in seen:
            continue
        seen.add(key)
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


def slice_size(w) -> int:
    """Distinct tasks in the calibration sample."""
    return min(w.n_tasks, max(SAMPLE_MIN, int(round(SLICE_FRACTION * w.n_tasks))))


def calibration_tasks(w, seed=0, sample=None):
    """Task indices of the calibration launch: a seeded sample, repeated to
    at least LAUNCH_MIN tasks."""
    rng = np.random.default_rng(seed)
    k = min(sample or slice_size(w), w.n_tasks)
    idx = np.sort(rng.choice(w.n_tasks, k, replace=False))
    reps = max(1, -(-LAUNCH_MIN // k))
    return np.tile(idx, reps)


def autotune(w, slice_tasks=None, seed=0, log=print):
    """Sweeps the tuning space on a calibration slice of w; returns (best,
    table of (ms, tuning))."""
    import paper_2001_10049_amd as xd
    sub = w.subset(calibration_tasks(w, seed, slice_tasks))
    store = xd.ReadStore.from_workload(sub)
    pairs, seeds, x = xd.workload_tensors(sub, "cuda")
    table = []
    for t in candidates(sub):
        ms = time_tuning(store, pairs, seeds, x, sub.k, t)
        table.append((ms, t))
        log("%8.3f ms  %s" % (ms, t))
    table.sort(key=lambda r: r[0])
    best = dict(table[0][1])
    # the band tier's workgroup count matters only when the slice reaches it
    xd.profile_enable(True)
    xd.profile_read(reset=True)
    time_tuning(store, pairs, seeds, x, sub.k, best, reps=1)
    prof = xd.profile_read(reset=True)
    xd.profile_enable(False)
    if prof["to_band"] > 0:
        band = []
        for bb in BAND_BLOCKS:
            t = dict(best, band_blocks=bb)
            ms = time_tuning(store, pairs, seeds, x, sub.k, t)
            band.append((ms, t))
            log("%8.3f ms  %s" % (ms, t))
        band.sort(key=lambda r: r[0])
        best = band[0][1]
        table += band
    store.close()
    return best, table


def main():
    ap = argparse.ArgumentParser(description="autotune the batched form")
    ap.add_argument("--workload", nargs="+", default=["c2", "c3"])
    ap.add_argument("--slice", type=int, default=0,
                    help="distinct calibration tasks (default: 1 %% of the workload, "
                    "at least %d), repeated to %d" % (SAMPLE_MIN, LAUNCH_MIN))
    ap.add_argument("--out", default=CACHE, help="where to write the merged cache")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    cache = _load_cache()
    dev = device_key()
    for name in args.workload:
        w = synth.config(name)
        t0 = time.time()
        best, table = autotune(w, args.slice or None,
                               log=lambda s: print(name, s, flush=True))
        entry = dict(best)
        entry["calibration_tasks"] = args.slice or slice_size(w)
        entry["calibration_launch"] = int(calibration_tasks(w, 0, args.slice or None).size)
        cache.setdefault(dev, {})[signature(w)] = entry
        print("%s %s -> %s (%.0f s)" % (name, signature(w), entry, time.time() - t0), flush=True)
    tmp = args.out + ".tmp"
    json.dump(cache, open(tmp, "w"), indent=1, sort_keys=True)
    os.replace(tmp, args.out)


if __name__ == "__main__":
    main()
