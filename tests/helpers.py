"""Small shared test helpers (inputs only; no alignment arithmetic)."""
import numpy as np

import synth

ACGT = "ACGT"


def rand_codes(rng, n):
    return rng.integers(0, 4, n, dtype=np.uint8)


def mutate_codes(rng, a, p=0.15):
    out = []
    for c in a:
        r = rng.random()
        if r < p / 3:
            continue
        if r < 2 * p / 3:
            out.append((int(c) + 1 + int(rng.integers(0, 3))) & 3)
        else:
            out.append(int(c))
        if rng.random() < p / 3:
            out.append(int(rng.integers(0, 4)))
    return np.array(out, np.uint8)


def workload_from(reads, tasks, k=17, name="explicit"):
    """reads: list of uint8 code arrays; tasks: list of (ra, rb, pa, pb, X)."""
    length = np.array([len(r) for r in reads], np.uint32)
    off = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.uint64)
    codes = np.concatenate(reads).astype(np.uint8) if reads else np.zeros(0, np.uint8)
    t = np.array(tasks, np.int64).reshape(-1, 5)
    n = t.shape[0]
    return synth.Workload(
        name=name, params={}, codes=codes, off=off, length=length,
        tspan=np.zeros((len(reads), 2), np.uint32),
        ra=t[:, 0].astype(np.uint32), rb=t[:, 1].astype(np.uint32),
        pa=t[:, 2].astype(np.uint32), pb=t[:, 3].astype(np.uint32),
        x=t[:, 4].astype(np.int32), ovl=np.zeros(n, np.uint32),
        spurious=np.zeros(n, np.uint8), k=k, n_candidate_pairs=n, n_candidate_tasks=n)
