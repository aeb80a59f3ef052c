"""Multi-seed pair alignment throughput (xd_align_pairs) on one MI355X.

Workload: every candidate pair of the c2/c3 read set (4.6 Mbp genome at 30x,
template overlap >= 1 kbp) with all of its true seeds kept >= 17 bp apart,
sorted by position in A, X = 25; every other pair is a reverse-strand twin (B
stored reverse-complemented and aligned with the reverse-complement flag).
The paper's three seed options (section 5) are timed: one seed per pair,
seeds >= 1 kbp apart, all seeds >= k apart.  One JSON line per option.

    python bench_pairs.py [--steps 3] [--warmup 1] [--cpu-pairs 300]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

OPTIONS = (("one-seed", 17, 1), ("1kbp-apart", 1000, 0), ("all-seeds-k-apart", 17, 0))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build(name="c3"):
    import numpy as np
    import synth
    from oracle.pairs import revcomp   # builds the reverse-strand copies of the input only
    w = synth.config(name, n_tasks=10 ** 8)   # every candidate (pair, seed) task
    a = np.minimum(w.ra, w.rb)
    b = np.maximum(w.ra, w.rb)
    flip = w.ra > w.rb
    pa = np.where(flip, w.pb, w.pa)
    pb = np.where(flip, w.pa, w.pb)
    order = np.lexsort((pb, pa, b, a))
    a, b, pa, pb = a[order], b[order], pa[order], pb[order]
    keys = a.astype(np.uint64) << 32 | b.astype(np.uint64)
    starts = np.concatenate([[0], np.nonzero(np.diff(keys))[0] + 1])
    n = starts.size
    seed_off = np.concatenate([starts, [keys.size]]).astype(np.uint64)
    ra, rb = a[starts].astype(np.uint32), b[starts].astype(np.uint32)
    rc = (np.arange(n) % 2).astype(np.uint8)
    codes, off, length = [w.codes], list(w.off), list(w.length)
    total, copy_of = int(w.codes.size), {}
    for p in np.nonzero(rc)[0]:
        r = int(rb[p])
        if r not in copy_of:
            seq = w.codes[int(w.off[r]):int(w.off[r]) + int(w.length[r])]
            codes.append(revcomp(seq))
            off.append(total)
            length.append(int(w.length[r]))
            total += int(w.length[r])
            copy_of[r] = len(length) - 1
        rb[p] = copy_of[r]
    return dict(codes=np.concatenate(codes), off=np.array(off, np.uint64),
                length=np.array(length, np.uint32), pairs=np.stack([ra, rb], 1), rc=rc,
                seed_off=seed_off, seeds=np.stack([pa, pb], 1).astype(np.uint32), k=w.k)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-pairs", type=int, default=300)
    args = ap.parse_args()
    import numpy as np
    import torch
    import paper_2001_10049_amd as xd
    log("building the pair lists")
    d = build()
    n, S = d["pairs"].shape[0], d["seeds"].shape[0]
    log("%d pairs, %d seeds, %d reverse-strand" % (n, S, int(d["rc"].sum())))
    store = xd.ReadStore(d["codes"], d["off"], d["length"])
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()  # noqa: E731
    pairs, seed_off = t(d["pairs"], np.int32), t(d["seed_off"], np.int64)
    seeds, rc = t(d["seeds"], np.int32), t(d["rc"], np.uint8)
    for name, md, mx in OPTIONS:
        run = lambda: xd.align_pairs(store, pairs, seed_off, seeds, rc=rc, x_scalar=25,  # noqa
                                     min_dist=md, max_seeds=mx, k=d["k"], n_seeds=S)
        for _ in range(args.warmup):
            out = run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        cells = int(out["cells"].sum())
        kept = int(out["n_kept"].sum())
        if int((out["status"] != 0).sum()):
            raise RuntimeError("pairs failed")
        line = {"metric": "multi-seed pair alignment (xd_align_pairs)", "option": name,
                "min_dist": md, "max_seeds": mx, "pairs": n, "seeds_listed": S,
                "seeds_aligned": kept, "ms_per_step": round(ms, 3),
                "gcups": round(cells / (ms / 1e3) / 1e9, 2),
                "pairs_per_s": round(n / (ms / 1e3), 1),
                "seeds_per_s": round(kept / (ms / 1e3), 1), "steps": args.steps,
                "dtype": "int32", "data": "synthetic",
                "config": {"workload": "c2/c3 read set: every candidate pair (template overlap "
                           ">= 1 kbp) with its true seeds >= 17 bp apart; X=25; every other "
                           "pair reverse-strand"}}
        if args.cpu_pairs and name == "one-seed":
            import oracle
            from oracle import pairs as op
            sel = np.arange(min(args.cpu_pairs, n))
            so = d["seed_off"]
            lo = np.concatenate([[0], np.cumsum(so[sel + 1] - so[sel])]).astype(np.uint64)
            sub_seeds = np.concatenate([d["seeds"][int(so[p]):int(so[p + 1])] for p in sel])
            threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
            t1 = time.perf_counter()
            r = op.align_pairs(d["codes"], d["off"], d["length"], d["pairs"][sel], lo, sub_seeds,
                               rc=d["rc"][sel], x_scalar=25, min_dist=md, max_seeds=mx,
                               k=d["k"], n_threads=threads)
            dt = time.perf_counter() - t1
            got = {k: v[:sel.size].cpu().numpy() for k, v in out.items()}
            assert np.array_equal(got["score"], r["score"]) and np.array_equal(
                got["cells"].view(np.uint64), r["cells"]), "GPU and oracle differ on the sample"
            line["cpu_baseline"] = {"value": round(int(r["cells"].sum()) / dt / 1e9, 3),
                                    "unit": "GCUPS", "cores": threads, "kind": "oracle",
                                    "pairs_per_s": round(sel.size / dt, 1),
                                    "sample": "first %d pairs, one-seed (%.1f s), results "
                                              "checked against the GPU's" % (sel.size, dt)}
        print(json.dumps(line), flush=True)
    store.close()


if __name__ == "__main__":
    main()
