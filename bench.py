#!/usr/bin/env python3
"""Benchmark: X-drop seed-and-extend throughput on one MI355X.

A step is one pass of the whole hot path over one batch: the seed score and
the left and right X-drop extensions of every task, all tiers and the
combine kernel (one xd_align_batch call).  The default workload is c2:
100,000 read pairs from a 30x synthetic 4.6 Mbp read set (log-normal
lengths, mean 10 kbp, sd 5 kbp, clipped 1-50 kbp; 5/5/5 % errors), one exact
17-mer seed per pair, X = 25, scores +1/-1/-1.  Inputs are resident in HBM
before the timed region; the read store upload is not timed.

Prints one JSON line: GCUPS (evaluated cells of both extensions per second,
the oracle's cell definition) as `value`, pairs/s beside it, the dominant
kernel's roofline position and the CPU oracle timed on a bounded sample
(all host threads, then one; the host CPU model).  Beside them: the batched
form's packed tier against the int32 and packed 16-bit peaks, the
2,000,000-task c3 workload (X in {7, 25, 50}) plain against batched, and a
short c5 serving window (Poisson requests, p50/p99 latency and pairs/s;
bench_serve.py runs the full 20 s window).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS and aligned pairs/sec for X-drop extension at X=25 (1 MI355X)"
# MI355X: 256 CUs x 64 int32 lanes per clock x 2.4 GHz
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
OPS_PER_CELL = 8  # compare, select, add diagonal, max(up,left), add gap, max, compare, select
KERNEL_NAMES = {"plain": "k_ext_first<1, 16, true>",
                "persistent": "k_pair_tier<4> (64-cell tier, two extensions per wave, queue)"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2.json")

WORKLOAD_DESC = {
    "c2": ("c2: 100,000 read pairs, 4.6 Mbp uniform genome at 30x, read lengths log-normal "
           "mean 10 kbp sd 5 kbp clipped 1-50 kbp, 5/5/5% sub/ins/del, one exact 17-mer seed "
           "per pair, X=25, +1/-1/-1"),
    "c1": ("c1: 1,000 read pairs, 200 kbp genome, reads 2-5 kbp, 5/5/5% errors, X=7, +1/-1/-1"),
    "c3": ("c3: 2,000,000 (pair, seed) tasks over the c2 read set (true seeds >= 17 apart), "
           "X uniform in {7, 25, 50}, +1/-1/-1"),
    "c4": ("c4: 20,000,000 (pair, seed) tasks, 100 Mbp genome (90 Mbp uniform + 2,000 copies "
           "of 200 random 5 kbp segments) at 30x, read lengths log-normal mean 12 kbp sd 6 kbp "
           "clipped 1-60 kbp, 4/4/4% errors, 10% of tasks from reads over different repeat "
           "copies, X=25, +1/-1/-1"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources the extension kernels and their launches are built from."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2001_10049_amd", "csrc")
    for f in ("xdrop.hip", "xdrop_device.h", "pair_device.h", "pair2_device.h", "pair4_device.h"):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch of the dominant kernel from committed counter runs,
    or None when the kernel sources changed since they were taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def xd_tuned(w):
    """Tuning for the batched forms: the autotuner's cached choice for this
    workload shape, else the library defaults."""
    try:
        from paper_2001_10049_amd import tune
        return tune.cached(w) or {}
    except Exception:
        return {}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds: float, threads: int | None = None):
    """The oracle as it stands, on the first tasks of w for about `seconds`."""
    import numpy as np
    import oracle
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    chunk = 2000 if threads > 1 else 200
    done = cells = 0
    t0 = time.perf_counter()
    while done < w.n_tasks and time.perf_counter() - t0 < seconds:
        idx = np.arange(done, min(done + chunk, w.n_tasks))
        res, used = oracle.align_batch(
            w.codes, w.off, w.length, np.stack([w.ra[idx], w.rb[idx]], 1),
            np.stack([w.pa[idx], w.pb[idx]], 1), x=w.x[idx], k=w.k, n_threads=threads)
        cells += int(res["cells"].sum())
        done += idx.size
    dt = time.perf_counter() - t0
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
            "kind": "oracle", "pairs_per_s": round(done / dt, 1),
            "sample": "first %d tasks of %s (%.1f s wall, %d cells)" % (done, w.name, dt, cells)}


def time_forms(xd, torch, w, forms, steps, warmup, tuning, dev, label):
    """Times each form on workload w (same output buffers, results checked
    equal across forms); returns (per-form results, profile of the first
    profiled form, cells per step)."""
    import numpy as np
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, dev)
    n = w.n_tasks
    out = dict(score=torch.empty(n, dtype=torch.int32, device=dev),
               beg=torch.empty((n, 2), dtype=torch.int32, device=dev),
               end=torch.empty((n, 2), dtype=torch.int32, device=dev),
               status=torch.empty(n, dtype=torch.int32, device=dev),
               cells=torch.empty(n, dtype=torch.int64, device=dev))
    plan = None
    if "plan" in forms:
        plan = xd.Plan(store, pairs, seeds, x=x, k=w.k, out=out, tuning=tuning)
    steppers = {
        "plain": lambda: xd.align_batch(store, pairs, seeds, x=x, k=w.k, out=out),
        "persistent": lambda: xd.align_batch(store, pairs, seeds, x=x, k=w.k, out=out,
                                             persistent=True, tuning=tuning),
        "plan": lambda: plan.launch(),
    }
    results, profs = {}, {}
    ref_out = None
    cells_per_step = 0
    for form in forms:
        step = steppers[form]
        log(label, "warmup", form, warmup)
        for _ in range(warmup):
            step()
        if form != "plan":
            xd.profile_enable(True)
            xd.profile_read(reset=True)
        log(label, "timing", form, steps, "steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p = xd.profile_read(reset=True) if form != "plan" else None
        xd.profile_enable(False)
        ms_f = (t1 - t0) * 1e3 / steps
        # every step computes the same results: check and count them now
        if int((out["status"] != 0).sum()) != 0:
            raise RuntimeError("tasks failed: %s" % np.unique(out["status"].cpu().numpy()))
        snap = {k: v.clone() for k, v in out.items()}
        if ref_out is None:
            ref_out = snap
        elif not all(torch.equal(ref_out[k], snap[k]) for k in snap):
            raise RuntimeError("form %s gave different results from %s" % (form, forms[0]))
        cells_per_step = int(out["cells"].sum())
        results[form] = {"ms_per_step": round(ms_f, 4),
                         "gcups": round(cells_per_step / (ms_f / 1e3) / 1e9, 2),
                         "pairs_per_s": round(n / (ms_f / 1e3), 1)}
        if p is not None:
            results[form]["ms_tier1_per_launch"] = round(p["ms_tier1"] / max(p["batches"], 1), 4)
            profs[form] = p
    if plan is not None:
        plan.close()
    store.close()
    del out, pairs, seeds, x
    torch.cuda.empty_cache()
    return results, profs, cells_per_step


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu1-seconds", type=float, default=6.0,
                    help="one-thread oracle sample (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--forms", default="plain,persistent,plan",
                    help="forms to time; the first one gives `value`")
    ap.add_argument("--tuning", default="",
                    help="JSON tuning for the batched forms (default: the tuned cache entry)")
    ap.add_argument("--c3-steps", type=int, default=3,
                    help="steps of the c3 plain-vs-batched comparison (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="measured window of the c5 serving run (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2001_10049_amd as xd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log("generating", args.workload)
    w = synth.config(args.workload)
    n = w.n_tasks
    tuning = json.loads(args.tuning) if args.tuning else xd_tuned(w)
    forms = [f for f in args.forms.split(",") if f]
    results, profs, cells_per_step = time_forms(xd, torch, w, forms, args.steps, args.warmup,
                                                tuning, dev, args.workload)
    head = forms[0]
    ms = results[head]["ms_per_step"]
    gcups = results[head]["gcups"]
    prof = profs.get(head) or next(iter(profs.values()))

    # dominant kernel: the 64-cell first tier; its algorithmic work is every
    # cell it completes (all cells when no extension moved to a wider tier)
    launches = max(prof["batches"], 1)
    if prof["to_tier2"] == 0 and (head == "plain" or w.x.max() <= 32):
        k_ms = prof["ms_tier1"] / launches
        kernel = KERNEL_NAMES.get(head, head)
    else:
        k_ms = (prof["ms_tier1"] + prof["ms_wide"]) / launches
        kernel = KERNEL_NAMES.get(head, head) + " + wide tiers"
    achieved = OPS_PER_CELL * cells_per_step / (k_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": round(PEAK_INT32_TOPS, 3), "unit": "TOP/s",
                "frac": round(achieved / PEAK_INT32_TOPS, 4), "traffic": load_traffic(),
                "kernel": kernel, "ms_per_launch": round(k_ms, 4),
                "cells_per_launch": cells_per_step, "ops_per_cell": OPS_PER_CELL,
                "kernel_gcups": round(cells_per_step / (k_ms / 1e3) / 1e9, 2),
                "ext_overflowed": [int(prof["to_tier2"]), int(prof["to_tier3"]),
                                   int(prof["to_tier4"]), int(prof["to_tier5"]),
                                   int(prof["to_band"])]}
    # the batched form's packed tier (two extensions per wave, 16-bit halves)
    # against both peaks: int32 lanes, and packed 16-bit lanes (twice that)
    # (only when that tier runs every extension: no X above its limit, no
    # overflow into the 128-cell tier)
    pp = profs.get("persistent")
    packed = None
    if pp is not None and pp["to_tier2"] == 0 and int(w.x.max()) <= tuning.get("x_tier1", 32):
        pk_ms = pp["ms_tier1"] / max(pp["batches"], 1)
        pk_ach = OPS_PER_CELL * cells_per_step / (pk_ms / 1e3) / 1e12
        packed = {"kernel": KERNEL_NAMES["persistent"], "ms_per_launch": round(pk_ms, 4),
                  "kernel_gcups": round(cells_per_step / (pk_ms / 1e3) / 1e9, 2),
                  "achieved": round(pk_ach, 3), "unit": "TOP/s",
                  "frac_int32_peak": round(pk_ach / PEAK_INT32_TOPS, 4),
                  "peak_packed16": round(2 * PEAK_INT32_TOPS, 3),
                  "frac_packed16_peak": round(pk_ach / (2 * PEAK_INT32_TOPS), 4)}

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # c3: batched (queue + persistent tiers, hipGraph plan) against plain on
    # the uneven 2,000,000-task workload
    c3 = None
    if args.c3_steps > 0 and args.workload != "c3":
        log("generating c3")
        w3 = synth.config("c3")
        r3, _, cells3 = time_forms(xd, torch, w3, ["plain", "persistent", "plan"],
                                   args.c3_steps, 1, xd_tuned(w3), dev, "c3")
        c3 = {"workload": WORKLOAD_DESC["c3"], "steps": args.c3_steps,
              "cells_per_step": cells3, "forms": r3,
              "batched_over_plain": round(r3["plan"]["gcups"] / r3["plain"]["gcups"], 3)}
        del w3

    serving = None
    if args.serve_seconds > 0:
        log("serving window (c5), %.0f s" % args.serve_seconds)
        import bench_serve
        serving = bench_serve.run(seconds=args.serve_seconds, warmup=1.0)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle), about %.0f s" % args.cpu_seconds)
        cpu = cpu_baseline(w, args.cpu_seconds)
        cpu["cpu_model"] = cpu_model()
        if args.cpu1_seconds > 0:
            log("cpu baseline, one thread, about %.0f s" % args.cpu1_seconds)
            one = cpu_baseline(w, args.cpu1_seconds, threads=1)
            cpu["one_thread"] = {"value": one["value"], "unit": "GCUPS",
                                 "pairs_per_s": one["pairs_per_s"], "sample": one["sample"]}

    rec = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC[args.workload], "pairs": n,
                   "form": head, "k": w.k, "tuning": tuning},
        "pairs_per_s": round(n / (ms / 1e3), 1),
        "forms": results,
        "cells_per_step": cells_per_step,
        "roofline": roofline,
        "packed_tier": packed,
        "c3": c3,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
