"""Candidate read pairs from shared retained k-mers: TEST INFRASTRUCTURE ONLY
(see oracle/__init__.py).

Section 2 of the paper drops k-mers that occur once across the reads
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
    stats dict(kmers, distinct, retained, occurrences, non_singletons))."""
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
    stats = dict(kmers=total, distinct=len(occ), retained=retained, occurrences=kept_occ,
                 non_singletons=sum(len(v) >= 2 for v in occ.values()))
    return pairs, seed_off, seeds, stats


def find_overlaps_sorted(codes, off, length, k=17, count_lo=2, count_hi=8):
    """The same result as find_overlaps, for read sets too large for a dict:
    all occurrences are ordered by k-mer code (a library sort), equal codes
    form each k-mer's list, and the pairs of every list of length
    count_lo..count_hi are generated list length by list length."""
    off = np.asarray(off, np.int64)
    length = np.asarray(length, np.int64)
    n_starts = np.maximum(length - k + 1, 0)
    total = int(n_starts.sum())
    code = np.empty(total, np.uint64)
    read = np.repeat(np.arange(len(length), dtype=np.uint32), n_starts)
    pos = np.empty(total, np.uint32)
    o = 0
    for r in np.nonzero(n_starts)[0]:
        n = int(n_starts[r])
        code[o:o + n] = kmer_codes(codes[int(off[r]):int(off[r]) + int(length[r])], k)
        pos[o:o + n] = np.arange(n, dtype=np.uint32)
        o += n
    order = np.argsort(code, kind="stable")
    code, read, pos = code[order], read[order], pos[order]
    del order
    start = np.flatnonzero(np.concatenate([[True], code[1:] != code[:-1]])) if total else \
        np.zeros(0, np.int64)
    count = np.diff(np.concatenate([start, [total]]))
    keep = (count >= count_lo) & (count <= count_hi)
    ra_l, rb_l, pa_l, pb_l = [], [], [], []
    for c in np.unique(count[keep]):
        s = start[keep & (count == c)]
        for x in range(c):
            for y in range(x + 1, c):
                a, b = s + x, s + y
                ra_l.append(read[a]); pa_l.append(pos[a])
                rb_l.append(read[b]); pb_l.append(pos[b])
    if ra_l:
        ra, rb = np.concatenate(ra_l), np.concatenate(rb_l)
        pa, pb = np.concatenate(pa_l), np.concatenate(pb_l)
    else:
        ra = rb = pa = pb = np.zeros(0, np.uint32)
    diff = ra != rb
    ra, rb, pa, pb = ra[diff], rb[diff], pa[diff], pb[diff]
    swap = ra > rb
    ra, rb = np.where(swap, rb, ra), np.where(swap, ra, rb)
    pa, pb = np.where(swap, pb, pa), np.where(swap, pa, pb)
    o = np.lexsort((pb, pa, rb, ra))
    ra, rb, pa, pb = ra[o], rb[o], pa[o], pb[o]
    head = np.flatnonzero(np.concatenate([[True], (ra[1:] != ra[:-1]) | (rb[1:] != rb[:-1])])) \
        if ra.size else np.zeros(0, np.int64)
    pairs = np.stack([ra[head], rb[head]], 1).astype(np.uint32).reshape(-1, 2)
    seed_off = np.concatenate([head, [ra.size]]).astype(np.uint64)
    seeds = np.stack([pa, pb], 1).astype(np.uint32).reshape(-1, 2)
    stats = dict(kmers=total, distinct=int(start.size), retained=int(keep.sum()),
                 occurrences=int(count[keep].sum()), non_singletons=int((count >= 2).sum()))
    return pairs, seed_off, seeds, stats
