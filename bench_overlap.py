"""Candidate-pair generation (xd_find_overlaps) on one MI355X, alone and
followed by the alignment of every candidate pair (xd_align_pairs).

Read set: workload c2's (13,743 reads, 138 Mbp, 30x of a 4.6 Mbp genome,
5/5/5 % errors); k = 17, m = 8.  Lines printed:
  overlap   k-mers per second through the whole stage (both filter passes,
            retention, pair expansion, sort, output), pairs and seeds found
  pipeline  candidates + alignment of every pair with one seed, and with all
            seeds at least k apart (X = 25, +1/-1/-1); ms and GCUPS
The oracle's sort-based form is timed on a sample of the reads.

    python bench_overlap.py [--steps 5] [--warmup 1] [--cpu-reads 1700] [--workload c2|c4]

--workload c4 runs the stage alone on c4's read set (250,273 reads, 3 Gbp, 30x
of a 100 Mbp genome with 10 % repeats, 12 % errors).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

K, M = 17, 8


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3 / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-reads", type=int, default=1700)
    ap.add_argument("--bloom-bits", type=int, default=0, help="first filter bits per k-mer")
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--workload", default="c2", choices=("c2", "c4"))
    args = ap.parse_args()
    import synth
    import paper_2001_10049_amd as xd
    w = synth.config(args.workload)
    if args.workload != "c2":
        args.no_pipeline = True
    store = xd.ReadStore.from_workload(w)
    bb = args.bloom_bits
    first = xd.find_overlaps(store, k=K, m=M, bloom_bits=bb)
    cap = (first["counts"]["pairs"], first["counts"]["seeds"])
    ov, ms = timed(lambda: xd.find_overlaps(store, k=K, m=M, bloom_bits=bb, capacity=cap),
                   args.steps, args.warmup)
    c = ov["counts"]
    line = {"metric": "candidate pairs (xd_find_overlaps): k-mers processed per second",
            "value": round(c["kmers"] / (ms / 1e3) / 1e6, 1), "unit": "M k-mers/s",
            "ms_per_step": round(ms, 3), "steps": args.steps, "warmup": args.warmup,
            "counts": c, "dtype": "u64 k-mer codes", "data": "synthetic",
            "config": {"workload": ("c2 read set: 13,743 reads, 138 Mbp, 30x of 4.6 Mbp, "
                                    "5/5/5 % errors" if args.workload == "c2" else
                                    "c4 read set: 250,273 reads, 3.0 Gbp, 30x of 100 Mbp with "
                                    "10 % repeats, 4/4/4 % errors") +
                       "; k = %d, retained counts 2..%d" % (K, M),
                       "bloom_bits": bb or 16}}
    if args.cpu_reads:
        from oracle import overlap as oov
        n = min(args.cpu_reads, w.length.size)
        t1 = time.perf_counter()
        r = oov.find_overlaps_sorted(w.codes, w.off[:n], w.length[:n], K, 2, M)
        dt = time.perf_counter() - t1
        line["cpu_baseline"] = {"value": round(r[3]["kmers"] / dt / 1e6, 2), "unit": "M k-mers/s",
                                "cores": 1, "kind": "oracle",
                                "sample": "first %d reads (%d k-mers, %.1f s), sort-based form"
                                          % (n, r[3]["kmers"], dt)}
    print(json.dumps(line), flush=True)

    for label, max_seeds in () if args.no_pipeline else (("one seed", 1),
                                                          ("all seeds k apart", 0)):
        def pipeline():
            o = xd.find_overlaps(store, k=K, m=M, bloom_bits=bb, capacity=cap)
            return xd.align_pairs(store, o["pairs"], o["seed_off"], o["seeds"], x_scalar=25,
                                  min_dist=K, max_seeds=max_seeds, k=K,
                                  n_seeds=o["counts"]["seeds"])
        out, ms2 = timed(pipeline, args.steps, args.warmup)
        cells = int(out["cells"].sum())
        kept = int(out["n_kept"].sum())
        if int((out["status"] != 0).sum()):
            raise RuntimeError("pairs failed to align")
        print(json.dumps({
            "metric": "candidates + alignment of every pair (%s)" % label,
            "ms_per_step": round(ms2, 3), "overlap_ms": round(ms, 3),
            "align_ms": round(ms2 - ms, 3), "pairs": c["pairs"], "alignments": kept,
            "gcups_alignment": round(cells / ((ms2 - ms) / 1e3) / 1e9, 1),
            "pairs_per_s": round(c["pairs"] / (ms2 / 1e3), 1), "dtype": "int32",
            "data": "synthetic",
            "config": {"workload": "c2 read set, k = %d, m = %d, X = 25, +1/-1/-1, seeds "
                       "selected at least k apart%s" % (K, M, ", first only" if max_seeds else "")}}),
            flush=True)
    store.close()


if __name__ == "__main__":
    main()
