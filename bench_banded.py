"""Banded Smith-Waterman throughput (xd_banded_batch) on one MI355X.

Workload c2 (100,000 read pairs from a 30x 4.6 Mbp read set, one true seed
each): each task aligns the two whole reads within w of the seed's diagonal.
One JSON line per band half-width; the oracle is timed on a sample.

    python bench_banded.py [--w 16 32 48] [--steps 5] [--warmup 1] [--cpu-tasks 300] [--trace]

With --trace each width also gets a line for xd_banded_traceback (the same
alignments plus begin cells and run-length paths).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
OPS_PER_CELL = 8  # diagonal add, floor of the diagonal neighbour, two maxes, floor, band select, ...


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--w", type=int, nargs="+", default=[16, 32, 48])
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-tasks", type=int, default=300)
    ap.add_argument("--trace", action="store_true", help="also time xd_banded_traceback")
    ap.add_argument("--max-ops", type=int, default=16384)
    ap.add_argument("--trace-budget", type=int, default=0, help="bytes (0: the library's)")
    args = ap.parse_args()
    import numpy as np
    import torch
    import synth
    import paper_2001_10049_amd as xd
    w = synth.config("c2")
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, _ = xd.workload_tensors(w, "cuda")
    for wd in args.w:
        run = lambda: xd.banded_batch(store, pairs, seeds, w_scalar=wd, k=w.k)  # noqa: E731
        for _ in range(args.warmup):
            out = run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        cells = int(out["cells"].sum())
        if int((out["status"] != 0).sum()):
            raise RuntimeError("tasks failed")
        gcups = cells / (ms / 1e3) / 1e9
        line = {"metric": "banded Smith-Waterman (xd_banded_batch)", "w": wd, "tasks": w.n_tasks,
                "ms_per_step": round(ms, 3), "gcups": round(gcups, 2),
                "pairs_per_s": round(w.n_tasks / (ms / 1e3), 1), "cells_per_step": cells,
                "roofline": {"bound": "alu", "achieved": round(OPS_PER_CELL * gcups / 1e3, 3),
                             "peak": round(PEAK_INT32_TOPS, 3), "unit": "TOP/s",
                             "frac": round(OPS_PER_CELL * gcups / 1e3 / PEAK_INT32_TOPS, 4)},
                "dtype": "int32", "data": "synthetic",
                "config": {"workload": "c2 read pairs (100,000, one true seed each), whole reads, "
                           "band |i - j - (pa - pb)| <= %d, +1/-1/-1" % wd}}
        if args.cpu_tasks and wd == args.w[-1]:
            import oracle
            idx = np.arange(min(args.cpu_tasks, w.n_tasks))
            t1 = time.perf_counter()
            r = oracle.banded_batch(w.codes, w.off, w.length, np.stack([w.ra, w.rb], 1)[idx],
                                    np.stack([w.pa, w.pb], 1)[idx], wd, k=w.k)
            dt = time.perf_counter() - t1
            got = out["score"][:idx.size].cpu().numpy()
            assert np.array_equal(got, r["score"]), "GPU and oracle differ on the sample"
            line["cpu_baseline"] = {"value": round(int(r["cells"].sum()) / dt / 1e9, 3),
                                    "unit": "GCUPS", "cores": 1, "kind": "oracle",
                                    "sample": "first %d tasks (%.1f s), scores checked against "
                                              "the GPU's" % (idx.size, dt)}
        print(json.dumps(line), flush=True)
        if args.trace:
            run_t = lambda: xd.banded_traceback(store, pairs, seeds, w_scalar=wd, k=w.k,  # noqa
                                                max_ops=args.max_ops,
                                                trace_budget=args.trace_budget)
            for _ in range(args.warmup):
                tr = run_t()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                tr = run_t()
            torch.cuda.synchronize()
            mst = (time.perf_counter() - t0) * 1e3 / args.steps
            if not torch.equal(tr["score"], out["score"]):
                raise RuntimeError("traced and untraced scores differ")
            n_ops = tr["n_ops"].cpu().numpy()
            print(json.dumps({
                "metric": "banded Smith-Waterman with traceback (xd_banded_traceback)", "w": wd,
                "tasks": w.n_tasks, "ms_per_step": round(mst, 3),
                "gcups": round(cells / (mst / 1e3) / 1e9, 2),
                "pairs_per_s": round(w.n_tasks / (mst / 1e3), 1),
                "ops_mean": round(float(n_ops.mean()), 1), "ops_max": int(n_ops.max()),
                "ops_over_capacity": int((n_ops > args.max_ops).sum()), "max_ops": args.max_ops,
                "trace_budget": args.trace_budget or "32 GiB",
                "dtype": "int32", "data": "synthetic",
                "config": line["config"]}), flush=True)
    store.close()


if __name__ == "__main__":
    main()
