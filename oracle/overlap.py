"""Candidate read pairs from shared retained k-mers: TEST INFRASTRUCTURE ONLY
(see oracle/__init__.py).

Section 3 of the paper drops k-mers that occur once across the reads
(singletons) and those occurring more than m times (likely repeats); the rest
are the retained k-mers.  Section 8 (Alg. 1) pairs every two entries of each
retained k-mer's list of (read, position) occurrences into an alignment task.
Readings: a k-mer's count is its number of occurrences (several in one read
count separately); retained means count_lo <= count <= count_hi (2 and m);
two occurrences in the same read make no task; k-mers are read on the forward
strand; the tasks are grouped per read pair (ra < rb) into the list of shared
positions (pa in ra, pb in rb), sorted.  Alg. 1's odd/even owner rule only
places tasks across ranks and has no counterpart on one GPU.
"""
from __future__ import annotations

import numpy as np


def kmer_codes(seq, k):
    """Integer code of every k-mer of seq (2 bits per base, first base highest)."""
    s = np.asarray(seq, np.uint64)
    n = s.size - k + 1
    if n <= 0:
        return np.zeros(0, np.uint64)
    code = np.zeros(n, np.uint64)
    for u in range(k):
        code = (code << np.uint64(2)) | s[u:u + n]
    return code


def find_overlaps(codes, off, length, k=17, count_lo=2, count_hi=8):
    """-> (pairs uint32[P, 2] sorted, seed_off uint64[P + 1], seeds uint32[S, 2],
    stats dict(kmers, distinct, retained, occurrences))."""
    occ = {}
    total = 0
    for r in range(len(length)):
        seq = codes[int(off[r]):int(off[r]) + int(length[r])]
        for p, key in enumerate(kmer_codes(seq, k).tolist()):
            occ.setdefault(key, []).append((r, p))
            total += 1
    per_pair = {}
    retained = kept_occ = 0
    for lst in occ.values():
        if not count_lo <= len(lst) <= count_hi:
            continue
        retained += 1
        kept_occ += len(lst)
        for x in range(len(lst)):
            for y in range(x + 1, len(lst)):
                (ra, pa), (rb, pb) = lst[x], lst[y]
                if ra == rb:
                    continue
                if ra > rb:
                    ra, pa, rb, pb = rb, pb, ra, pa
                per_pair.setdefault((ra, rb), []).append((pa, pb))
    keys = sorted(per_pair)
    pairs = np.array(keys, np.uint32).reshape(-1, 2)
    lists = [sorted(per_pair[key]) for key in keys]
    seed_off = np.concatenate([[0], np.cumsum([len(l) for l in lists])]).astype(np.uint64)
    seeds = (np.array([s for l in lists for s in l], np.uint32).reshape(-1, 2) if lists
             else np.zeros((0, 2), np.uint32))
    stats = dict(kmers=total, distinct=len(occ), retained=retained, occurrences=kept_occ)
    return pairs, seed_off, seeds, stats
