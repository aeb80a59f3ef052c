"""Records the oracle's results for every task of the large workload recipes
as chunked digests (tests/golden/oracle_digests.json), so that GPU tests can
check every task without rerunning the oracle.  Calls only the oracle and the
seeded generator.

    python tests/golden/make_oracle_digests.py c2 c3 c4 c5 [--threads 8]

Each finished chunk is kept in oracle_digests.json.<name>.partial until the
workload is recorded, so an interrupted run resumes where it stopped.
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
        # chunk records survive an interruption: a rerun resumes after the
        # last finished chunk of the same inputs
        part_path = args.out + "." + name + ".partial"
        inp = input_digest(w)
        try:
            part = json.load(open(part_path))
            if part.get("input") != inp:
                part = None
        except (OSError, ValueError):
            part = None
        if part is None:
            part = {"input": inp, "chunks": [], "cells": 0, "score_sum": 0, "status_nonzero": 0}
        for lo in range(len(part["chunks"]) * CHUNK, w.n_tasks, CHUNK):
            idx = np.arange(lo, min(lo + CHUNK, w.n_tasks))
            r = oracle.align_workload(w.subset(idx), n_threads=args.threads)
            part["chunks"] += result_digests(r)
            part["cells"] += int(r["cells"].astype(np.uint64).sum())
            part["score_sum"] += int(r["score"].astype(np.int64).sum())
            part["status_nonzero"] += int((r["status"] != 0).sum())
            json.dump(part, open(part_path + ".tmp", "w"))
            os.replace(part_path + ".tmp", part_path)
            print("%s: tasks %d..%d done (%.0f s)" % (name, lo, idx[-1], time.time() - t0),
                  flush=True)
        entry = {"input": inp, "tasks": int(w.n_tasks), "chunk": CHUNK,
                 "chunks": part["chunks"], "cells": part["cells"],
                 "score_sum": part["score_sum"], "status_nonzero": part["status_nonzero"]}
        try:
            db = json.load(open(args.out))
        except (OSError, ValueError):
            db = {}
        db[name] = entry
        tmp = args.out + ".tmp"
        json.dump(db, open(tmp, "w"), indent=1, sort_keys=True)
        os.replace(tmp, args.out)
        os.remove(part_path)
        print("%s: recorded (%.0f s)" % (name, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
