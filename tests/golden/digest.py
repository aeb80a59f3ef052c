"""Chunked SHA-256 digests of a workload's inputs and of per-task results.

Shared by the script that records the oracle's results
(make_oracle_digests.py) and the GPU tests that compare against them; it
holds no alignment arithmetic."""
import hashlib

import numpy as np

CHUNK = 100_000


def input_digest(w) -> str:
    h = hashlib.sha256()
    for a in (w.codes, w.length, w.ra, w.rb, w.pa, w.pb, w.x):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:32]


def result_digests(res, chunk=CHUNK):
    """res: score, beg, end, status, cells (any integer dtypes of those widths)."""
    score = np.ascontiguousarray(res["score"]).view(np.int32)
    beg = np.ascontiguousarray(res["beg"]).view(np.uint32).reshape(-1, 2)
    end = np.ascontiguousarray(res["end"]).view(np.uint32).reshape(-1, 2)
    status = np.ascontiguousarray(res["status"]).view(np.int32)
    cells = np.ascontiguousarray(res["cells"]).view(np.uint64)
    out = []
    for lo in range(0, score.shape[0], chunk):
        hi = lo + chunk
        h = hashlib.sha256()
        for a in (score[lo:hi], beg[lo:hi], end[lo:hi], status[lo:hi], cells[lo:hi]):
            h.update(np.ascontiguousarray(a).tobytes())
        out.append(h.hexdigest()[:24])
    return out


def reads_digest(w) -> str:
    """Digest of a workload's read set alone (bases and lengths)."""
    h = hashlib.sha256()
    for a in (w.codes, w.length):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:32]


def overlap_digest(pairs, seed_off, seeds) -> str:
    """Digest of a candidate-pair result: pairs uint32[P, 2], seed_off
    uint64[P + 1], seeds uint32[S, 2] (any integer dtypes of those widths)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pairs).view(np.uint32).tobytes())
    h.update(np.ascontiguousarray(seed_off).view(np.uint64).tobytes())
    h.update(np.ascontiguousarray(seeds).view(np.uint32).tobytes())
    return h.hexdigest()[:32]
