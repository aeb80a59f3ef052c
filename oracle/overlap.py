"""Candidate read pairs from shared retained k-mers: TEST INFRASTRUCTURE ONLY
(see oracle/__init__.py).

Section 2 of the paper drops k-mers that occur once across the reads
(singletons) and those occurring more than m times (likely repeats); the rest
are the retained k-mers.  Section 8 (Alg. 1) pairs every two entries of each
retained k-mer's list of (read, position) occurrences into an alignment task.
Readings: a k-mer's count is its number of occurrences (several in one read
count separately); retained means count_lo <= count <= count_hi (2 and m);
two occurrences in the same read make no task; the tasks are grouped per read
pair (ra < rb) into the list of shared positions (pa in ra, pb in rb),
sorted.  Alg. 1's odd/even owner rule only places tasks across ranks and has
no counterpart on one GPU.

Strand (the paper does not discuss it).  strands=1 reads k-mers on the
forward strand only.  strands=2 reads both: each occurrence counts under its
canonical k-mer, the smaller of its code and its reverse complement's code,
with a strand bit (1 when the reverse complement is the smaller).  Two
occurrences of a canonical k-mer with equal strand bits pair as above
(rc = 0); with different bits read rb matches the reverse complement of read
ra there (rc = 1), and the seed is (pa, len(rb) - k - pb): pb counted in
rb' = the reverse complement of rb, the coordinates xd_align_pairs takes for
a reverse-strand pair.  A k-mer equal to its own reverse complement (even k
only) has strand bit 0 everywhere, so its occurrences pair only with rc = 0.
Pairs are then keyed (ra, rb, rc) and sorted that way.
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


def revcomp_codes(code, k):
    """Code of the reverse complement of every k-mer code (base b -> 3 - b,
    order reversed)."""
    code = np.asarray(code, np.uint64)
    out = np.zeros(code.shape, np.uint64)
    for u in range(k):
        base = (code >> np.uint64(2 * u)) & np.uint64(3)
        out = (out << np.uint64(2)) | (np.uint64(3) - base)
    return out


def occurrences(seq, k, strands):
    """(code, strand bit) of every k-mer start of seq: the forward code and
    bit 0 (strands=1), or the canonical code and its strand bit (strands=2)."""
    f = kmer_codes(seq, k)
    if strands == 1:
        return f, np.zeros(f.size, np.uint8)
    r = revcomp_codes(f, k)
    return np.minimum(f, r), (r < f).astype(np.uint8)


def find_overlaps(codes, off, length, k=17, count_lo=2, count_hi=8, strands=1):
    """-> (pairs uint32[P, 2] sorted, seed_off uint64[P + 1], seeds uint32[S, 2],
    stats dict(kmers, distinct, retained, occurrences, non_singletons)), and
    with strands=2 a fifth item: rc uint8[P]."""
    assert strands in (1, 2)
    occ = {}
    total = 0
    for r in range(len(length)):
        seq = codes[int(off[r]):int(off[r]) + int(length[r])]
        code, sbit = occurrences(seq, k, strands)
        for p, (key, sb) in enumerate(zip(code.tolist(), sbit.tolist())):
            occ.setdefault(key, []).append((r, p, sb))
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
                (ra, pa, sa), (rb, pb, sb) = lst[x], lst[y]
                if ra == rb:
                    continue
                if ra > rb:
                    ra, pa, rb, pb = rb, pb, ra, pa
                rc = sa ^ sb
                if rc:
                    pb = int(length[rb]) - k - pb
                per_pair.setdefault((ra, rb, rc), []).append((pa, pb))
    keys = sorted(per_pair)
    pairs = np.array([key[:2] for key in keys], np.uint32).reshape(-1, 2)
    rcs = np.array([key[2] for key in keys], np.uint8)
    lists = [sorted(per_pair[key]) for key in keys]
    seed_off = np.concatenate([[0], np.cumsum([len(l) for l in lists])]).astype(np.uint64)
    seeds = (np.array([s for l in lists for s in l], np.uint32).reshape(-1, 2) if lists
             else np.zeros((0, 2), np.uint32))
    stats = dict(kmers=total, distinct=len(occ), retained=retained, occurrences=kept_occ,
                 non_singletons=sum(len(v) >= 2 for v in occ.values()))
    if strands == 2:
        return pairs, seed_off, seeds, stats, rcs
    return pairs, seed_off, seeds, stats


def find_overlaps_sorted(codes, off, length, k=17, count_lo=2, count_hi=8, strands=1):
    """The same result as find_overlaps, for read sets too large for a dict:
    all occurrences are ordered by k-mer code (a library sort), equal codes
    form each k-mer's list, and the pairs of every list of length
    count_lo..count_hi are generated list length by list length."""
    assert strands in (1, 2)
    off = np.asarray(off, np.int64)
    length = np.asarray(length, np.int64)
    n_starts = np.maximum(length - k + 1, 0)
    total = int(n_starts.sum())
    code = np.empty(total, np.uint64)
    sbit = np.empty(total, np.uint8)
    read = np.repeat(np.arange(len(length), dtype=np.uint32), n_starts)
    pos = np.empty(total, np.uint32)
    o = 0
    for r in np.nonzero(n_starts)[0]:
        n = int(n_starts[r])
        code[o:o + n], sbit[o:o + n] = occurrences(
            codes[int(off[r]):int(off[r]) + int(length[r])], k, strands)
        pos[o:o + n] = np.arange(n, dtype=np.uint32)
        o += n
    order = np.argsort(code, kind="stable")
    code, read, pos, sbit = code[order], read[order], pos[order], sbit[order]
    del order
    start = np.flatnonzero(np.concatenate([[True], code[1:] != code[:-1]])) if total else \
        np.zeros(0, np.int64)
    count = np.diff(np.concatenate([start, [total]]))
    keep = (count >= count_lo) & (count <= count_hi)
    ra_l, rb_l, pa_l, pb_l, rc_l = [], [], [], [], []
    for c in np.unique(count[keep]):
        s = start[keep & (count == c)]
        for x in range(c):
            for y in range(x + 1, c):
                a, b = s + x, s + y
                ra_l.append(read[a]); pa_l.append(pos[a])
                rb_l.append(read[b]); pb_l.append(pos[b])
                rc_l.append(sbit[a] ^ sbit[b])
    if ra_l:
        ra, rb = np.concatenate(ra_l), np.concatenate(rb_l)
        pa, pb = np.concatenate(pa_l), np.concatenate(pb_l)
        rc = np.concatenate(rc_l)
    else:
        ra = rb = pa = pb = np.zeros(0, np.uint32)
        rc = np.zeros(0, np.uint8)
    diff = ra != rb
    ra, rb, pa, pb, rc = ra[diff], rb[diff], pa[diff], pb[diff], rc[diff]
    swap = ra > rb
    ra, rb = np.where(swap, rb, ra), np.where(swap, ra, rb)
    pa, pb = np.where(swap, pb, pa), np.where(swap, pa, pb)
    # a reverse-strand seed counts pb in the reverse complement of read rb
    pb = np.where(rc == 1, length[rb] - k - pb.astype(np.int64), pb).astype(np.uint32)
    o = np.lexsort((pb, pa, rc, rb, ra))
    ra, rb, pa, pb, rc = ra[o], rb[o], pa[o], pb[o], rc[o]
    head = np.flatnonzero(np.concatenate(
        [[True], (ra[1:] != ra[:-1]) | (rb[1:] != rb[:-1]) | (rc[1:] != rc[:-1])])) \
        if ra.size else np.zeros(0, np.int64)
    pairs = np.stack([ra[head], rb[head]], 1).astype(np.uint32).reshape(-1, 2)
    seed_off = np.concatenate([head, [ra.size]]).astype(np.uint64)
    seeds = np.stack([pa, pb], 1).astype(np.uint32).reshape(-1, 2)
    stats = dict(kmers=total, distinct=int(start.size), retained=int(keep.sum()),
                 occurrences=int(count[keep].sum()), non_singletons=int((count >= 2).sum()))
    if strands == 2:
        return pairs, seed_off, seeds, stats, rc[head].astype(np.uint8)
    return pairs, seed_off, seeds, stats
