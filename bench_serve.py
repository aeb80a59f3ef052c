#!/usr/bin/env python3
"""Serving benchmark (c5): Poisson arrivals of alignment requests against a
resident read store; reports p50/p99 latency beside pairs/s and GCUPS.

Store: 30x synthetic 4.6 Mbp read set, read lengths log-normal (mean 10 kbp,
sd 5 kbp) clipped to 1-100 kbp, 5/5/5 % errors.  Requests: sizes log-uniform
integers on [1, 10,000] pairs drawn from the set's true (pair, seed) tasks,
X from {7, 25} per request, arrivals Poisson at --rate per second.  Latency
is from submission to results in host memory, on the server's clock.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--rate", type=float, default=2000.0, help="requests per second")
    ap.add_argument("--seconds", type=float, default=20.0, help="measured window")
    ap.add_argument("--warmup", type=float, default=2.0, help="arrivals before the window")
    ap.add_argument("--max-size", type=int, default=10000)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--budget-mib", type=int, default=2048)
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--max-batch", type=int, default=65536)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        print("needs a GPU", file=sys.stderr)
        sys.exit(2)
    print(json.dumps(run(**{k: v for k, v in vars(args).items()})), flush=True)


def run(rate=2000.0, seconds=20.0, warmup=2.0, max_size=10000, workload="c5", budget_mib=2048,
        slots=3, max_batch=65536, seed=7) -> dict:
    """One serving run; returns the JSON record."""
    args = argparse.Namespace(rate=rate, seconds=seconds, warmup=warmup, max_size=max_size,
                              workload=workload, budget_mib=budget_mib, slots=slots,
                              max_batch=max_batch, seed=seed)
    import numpy as np
    import synth
    import paper_2001_10049_amd as xd

    print("generating", args.workload, file=sys.stderr, flush=True)
    w = synth.config(args.workload)
    store = xd.ReadStore.from_workload(w)
    rng = np.random.default_rng(args.seed)
    total_s = args.warmup + args.seconds
    n_req = int(rng.poisson(args.rate * total_s))
    arrivals = np.sort(rng.uniform(0, total_s, n_req))
    sizes = np.minimum(np.floor(np.exp(rng.uniform(0, np.log(args.max_size + 1), n_req))),
                       args.max_size).astype(np.int64)
    sizes = np.maximum(sizes, 1)
    starts = rng.integers(0, w.n_tasks - args.max_size, n_req)
    xs = rng.choice([7, 25], n_req)
    pairs_all = np.stack([w.ra, w.rb], 1)
    seeds_all = np.stack([w.pa, w.pb], 1)
    tuning = {}
    try:
        from paper_2001_10049_amd import tune
        tuning = tune.cached(w) or {}
    except Exception:
        pass
    srv = xd.Server(store, hbm_budget_bytes=args.budget_mib << 20, slots=args.slots,
                    max_batch_tasks=args.max_batch, k=w.k, tuning=tuning)
    ids = [None] * n_req
    results = [None] * n_req
    done = threading.Event()

    def collector():
        for q in range(n_req):
            while ids[q] is None:
                time.sleep(0.0002)
            r = srv.poll(ids[q], timeout_ms=-1)
            results[q] = (r["info"], int(r["cells"].sum()), int((r["status"] != 0).sum()))
        done.set()

    th = threading.Thread(target=collector, daemon=True)
    th.start()
    print("submitting %d requests over %.1f s" % (n_req, total_s), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for q in range(n_req):
        while True:
            dt = arrivals[q] - (time.perf_counter() - t0)
            if dt <= 0:
                break
            if dt > 0.0005:
                time.sleep(dt - 0.0003)
        s = int(starts[q])
        n = int(sizes[q])
        ids[q] = srv.submit(pairs_all[s:s + n], seeds_all[s:s + n], x_scalar=int(xs[q]))
    done.wait()
    st = srv.stats()
    srv.close()
    store.close()
    # steady window: requests that arrived after the warm-up
    win = arrivals >= args.warmup
    lat = np.array([results[q][0]["t_done"] - results[q][0]["t_submit"]
                    for q in range(n_req)])[win]
    # the two parts of a latency: waiting for admission, then the batch
    wait = np.array([results[q][0]["t_start"] - results[q][0]["t_submit"]
                     for q in range(n_req)])[win]
    run_t = lat - wait
    t_first = min(results[q][0]["t_submit"] for q in range(n_req) if win[q])
    t_last = max(results[q][0]["t_done"] for q in range(n_req) if win[q])
    span = t_last - t_first
    pairs = int(sizes[win].sum())
    cells = sum(results[q][1] for q in range(n_req) if win[q])
    bad = sum(results[q][2] for q in range(n_req))
    rec = {
        "metric": "serving latency and throughput (c5)", "unit": "ms",
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "mean_ms": round(float(lat.mean()) * 1e3, 3),
        "wait_p50_ms": round(float(np.percentile(wait, 50)) * 1e3, 3),
        "wait_p99_ms": round(float(np.percentile(wait, 99)) * 1e3, 3),
        "batch_p50_ms": round(float(np.percentile(run_t, 50)) * 1e3, 3),
        "batch_p99_ms": round(float(np.percentile(run_t, 99)) * 1e3, 3),
        "pairs_per_s": round(pairs / span, 1), "gcups": round(cells / span / 1e9, 2),
        "offered_pairs_per_s": round(float(sizes[win].sum()) / args.seconds, 1),
        "requests": int(win.sum()), "rate": args.rate, "failed_tasks": bad,
        "batches": st["batches"], "peak_busy_slots": st["peak_busy_slots"],
        "peak_inflight_mib": round(st["peak_inflight_bytes"] / 2**20, 1),
        "budget_mib": args.budget_mib, "slots": args.slots,
        "config": {"workload": "c5: 30x 4.6 Mbp store, reads 1-100 kbp log-normal; request "
                   "sizes log-uniform 1-%d; X in {7, 25}; Poisson %.0f req/s; %.1f s window"
                   % (args.max_size, args.rate, args.seconds)},
        "data": "synthetic",
    }
    return rec


if __name__ == "__main__":
    main()
