"""Multi-seed pair alignment: TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Per candidate pair the paper explores a subset of its shared k-mers as seeds
(section 5: one seed per pair, all seeds at least the k-mer length apart, or
seeds 1,000 bp apart; section 8: a minimum distance between seeds and a maximum
number of seeds per overlap), aligns from each, and the pair's alignment is
the best of them.  Reads may overlap on opposite strands; then B is aligned
reverse-complemented.  Plain Python over the pinned task oracle.

Readings (the paper gives the options, not the procedure): seeds are chosen by
scanning the pair's list in order (normally increasing position in A) and
keeping a seed when it is the first kept one or lies at least min_dist past
the last kept seed in A, until max_seeds are kept (0 = no limit); the pair's
result is its best kept seed by score, the earliest kept on ties; for a
reverse-complement pair, B' = complement of B read backwards, and the seed
position in B and the result coordinates for B are positions in B'.
"""
from __future__ import annotations

import numpy as np

from . import TASK_OK, align_batch

TASK_NO_SEED = 5   # the pair's seed list is empty
NO_SEED_IDX = 0xFFFFFFFF


def revcomp(codes) -> np.ndarray:
    """Reverse complement of a code string (A=0 C=1 G=2 T=3, so complement = 3 - c)."""
    c = np.asarray(codes, np.uint8)
    return (3 - c[::-1]).astype(np.uint8)


def select_seeds(pa, min_dist: int, max_seeds: int):
    """Indices into pa of the seeds kept (rule in the module docstring)."""
    kept = []
    last = None
    for i, p in enumerate(int(v) for v in pa):
        if max_seeds and len(kept) >= max_seeds:
            break
        if last is None or p >= last + min_dist:
            kept.append(i)
            last = p
    return kept


def align_pairs(codes, off, length, pairs, seed_off, seeds, rc=None, x=None, x_scalar=0,
                min_dist=17, max_seeds=0, k=17, match=1, mismatch=-1, gap=-1, n_threads=None):
    """Per pair: select seeds, align each (B reverse-complemented when rc),
    keep the best.  pairs uint32[n, 2]; seed_off uint64[n + 1]; seeds
    uint32[S, 2] as (pa, pb); rc uint8[n] or None; x int32[n] or None.
    Returns dict of per-pair arrays: score, beg[n, 2], end[n, 2], status,
    seed_idx (index in the pair's list), n_kept, cells."""
    codes = np.ascontiguousarray(codes, np.uint8)
    off = np.asarray(off, np.uint64)
    length = np.asarray(length, np.uint32)
    pairs = np.asarray(pairs, np.uint32).reshape(-1, 2)
    seed_off = np.asarray(seed_off, np.uint64)
    seeds = np.asarray(seeds, np.uint32).reshape(-1, 2)
    n = pairs.shape[0]
    rc = np.zeros(n, np.uint8) if rc is None else np.asarray(rc, np.uint8)
    # reverse-complemented copies of the B reads of rc pairs, appended
    extra, copy_of = [], {}
    base = int(codes.size)
    n_reads = int(length.size)
    new_off, new_len = list(off), list(length)
    for p in range(n):
        b = int(pairs[p, 1])
        if rc[p] and b < n_reads and b not in copy_of:
            seq = codes[int(off[b]):int(off[b]) + int(length[b])]
            copy_of[b] = n_reads + len(extra)
            extra.append(revcomp(seq))
            new_off.append(base)
            new_len.append(int(length[b]))
            base += int(length[b])
    all_codes = np.concatenate([codes] + extra) if extra else codes
    all_off = np.array(new_off, np.uint64)
    all_len = np.array(new_len, np.uint32)
    # one task per kept seed
    t_pairs, t_seeds, t_x, owner, idx_in_list = [], [], [], [], []
    kept_count = np.zeros(n, np.uint32)
    for p in range(n):
        lo, hi = int(seed_off[p]), int(seed_off[p + 1])
        kept = select_seeds(seeds[lo:hi, 0], min_dist, max_seeds)
        kept_count[p] = len(kept)
        a, b = int(pairs[p, 0]), int(pairs[p, 1])
        if rc[p] and b < n_reads:
            b = copy_of[b]
        for i in kept:
            t_pairs.append((a, b))
            t_seeds.append(tuple(int(v) for v in seeds[lo + i]))
            t_x.append(int(x[p]) if x is not None else int(x_scalar))
            owner.append(p)
            idx_in_list.append(i)
    out = dict(score=np.full(n, np.iinfo(np.int32).min, np.int32),
               beg=np.zeros((n, 2), np.uint32), end=np.zeros((n, 2), np.uint32),
               status=np.full(n, TASK_NO_SEED, np.int32),
               seed_idx=np.full(n, NO_SEED_IDX, np.uint32), n_kept=kept_count,
               cells=np.zeros(n, np.uint64))
    if not t_pairs:
        return out
    res, _ = align_batch(all_codes, all_off, all_len, np.array(t_pairs, np.uint32),
                         np.array(t_seeds, np.uint32), x=np.array(t_x, np.int32), k=k,
                         match=match, mismatch=mismatch, gap=gap, n_threads=n_threads)
    seen = np.zeros(n, bool)
    for t, p in enumerate(owner):
        out["cells"][p] += res["cells"][t]
        if not seen[p]:  # the first kept seed fixes the status until one aligns
            out["status"][p] = res["status"][t]
            seen[p] = True
        if res["status"][t] != TASK_OK:
            continue
        if out["status"][p] != TASK_OK or res["score"][t] > out["score"][p]:
            out["status"][p] = TASK_OK
            out["score"][p] = res["score"][t]
            out["beg"][p] = res["beg"][t]
            out["end"][p] = res["end"][t]
            out["seed_idx"][p] = idx_in_list[t]
    return out
