"""Records the oracle's results for every task of the large workload recipes
as chunked digests (tests/golden/oracle_digests.json), so that GPU tests can
check every task without rerunning the oracle.  Calls only the oracle and the
seeded generator.

    python tests/golden/make_oracle_digests.py c2 c3 c5 [--threads 8]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from digest import CHUNK, input_digest, result_digests  # noqa: E402

OUT = os.path.join(HERE, "oracle_digests.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    for name in args.configs:
        t0 = time.time()
        w = synth.config(name)
        print("%s: %d tasks, generated in %.0f s" % (name, w.n_tasks, time.time() - t0), flush=True)
        parts = {k: [] for k in ("score", "beg", "end", "status", "cells")}
        for lo in range(0, w.n_tasks, CHUNK):
            idx = np.arange(lo, min(lo + CHUNK, w.n_tasks))
            r = oracle.align_workload(w.subset(idx), n_threads=args.threads)
            for k in parts:
                parts[k].append(r[k])
            print("%s: tasks %d..%d done (%.0f s)" % (name, lo, idx[-1], time.time() - t0),
                  flush=True)
        res = {k: np.concatenate(v) for k, v in parts.items()}
        entry = {"input": input_digest(w), "tasks": int(w.n_tasks), "chunk": CHUNK,
                 "chunks": result_digests(res), "cells": int(res["cells"].sum()),
                 "score_sum": int(res["score"].astype(np.int64).sum()),
                 "status_nonzero": int((res["status"] != 0).sum())}
        try:
            db = json.load(open(args.out))
        except (OSError, ValueError):
            db = {}
        db[name] = entry
        tmp = args.out + ".tmp"
        json.dump(db, open(tmp, "w"), indent=1, sort_keys=True)
        os.replace(tmp, args.out)
        print("%s: recorded (%.0f s)" % (name, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
