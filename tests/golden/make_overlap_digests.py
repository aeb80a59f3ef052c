"""Records the oracle's candidate pairs for whole read sets.

For each named workload's read set this runs oracle.overlap's sort-based
form (whose equality with the plain dict form is pinned in
tests/test_oracle_overlap.py) and stores the counts and a digest of the full
result in overlap_digests.json.  It calls nothing but the oracle and the
seeded generator.  Usage: python tests/golden/make_overlap_digests.py c2-small c2
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import synth  # noqa: E402
from digest import overlap_digest, reads_digest  # noqa: E402
from oracle import overlap as ov  # noqa: E402

K, M = 17, 8
OUT = os.path.join(HERE, "overlap_digests.json")


def main(names):
    rec = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.time()
        w = synth.config(name)
        pairs, seed_off, seeds, st = ov.find_overlaps_sorted(w.codes, w.off, w.length, K, 2, M)
        rec[name] = dict(k=K, m=M, reads=reads_digest(w), digest=overlap_digest(pairs, seed_off, seeds),
                         pairs=int(pairs.shape[0]), seeds=int(seeds.shape[0]),
                         **{f: int(st[f]) for f in ("kmers", "non_singletons", "retained",
                                                    "occurrences")})
        print("%s: %d pairs, %d seeds (%.0f s)" % (name, pairs.shape[0], seeds.shape[0],
                                                   time.time() - t0), flush=True)
        json.dump(rec, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
