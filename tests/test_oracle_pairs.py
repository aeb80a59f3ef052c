"""Pins for the multi-seed pair oracle (oracle/pairs.py): seed selection
against its defining properties, the reverse complement, the best-per-pair
rule and the reverse-strand closed form."""
import numpy as np
import pytest

import oracle
from oracle import pairs as op

from helpers import rand_codes


def test_revcomp_hand_and_involution():
    # ACGTT -> complement TGCAA -> reversed AACGT
    assert op.revcomp(np.array([0, 1, 2, 3, 3], np.uint8)).tolist() == [0, 0, 1, 2, 3]
    rng = np.random.default_rng(1)
    a = rand_codes(rng, 1001)
    assert np.array_equal(op.revcomp(op.revcomp(a)), a)
    assert op.revcomp(np.zeros(0, np.uint8)).size == 0


def test_select_hand_cases():
    pa = [0, 5, 17, 30, 34, 1000, 1016, 1017]
    assert op.select_seeds(pa, 17, 0) == [0, 2, 4, 5, 7]
    assert op.select_seeds(pa, 17, 2) == [0, 2]
    assert op.select_seeds(pa, 1000, 0) == [0, 5]
    assert op.select_seeds(pa, 17, 1) == [0]
    assert op.select_seeds(pa, 0, 0) == list(range(8))
    assert op.select_seeds([], 17, 0) == []


def _is_greedy_selection(pa, kept, min_dist, max_seeds):
    """Checks the defining properties instead of replaying the scan: kept
    indices increase, start at 0, are min_dist apart in pa; every index
    skipped before the last kept one, or after it while the limit is not
    reached, is closer than min_dist to the kept seed before it."""
    if not len(pa):
        return kept == []
    if kept[:1] != [0] or sorted(set(kept)) != kept:
        return False
    if max_seeds and len(kept) > max_seeds:
        return False
    for u, v in zip(kept, kept[1:]):
        if pa[v] < pa[u] + min_dist:
            return False
    scan_end = len(pa) if not (max_seeds and len(kept) == max_seeds) else kept[-1] + 1
    for i in range(scan_end):
        if i in kept:
            continue
        prev = max(j for j in kept if j < i)
        if pa[i] >= pa[prev] + min_dist:
            return False
    return True


@pytest.mark.parametrize("seed", range(6))
def test_select_properties_random(seed):
    rng = np.random.default_rng(seed)
    for _ in range(200):
        n = int(rng.integers(0, 25))
        pa = np.sort(rng.integers(0, 300, n)).tolist()
        md = int(rng.choice([0, 1, 17, 50]))
        mx = int(rng.choice([0, 1, 3]))
        kept = op.select_seeds(pa, md, mx)
        assert _is_greedy_selection(pa, kept, md, mx), (pa, md, mx, kept)


def _reads(*seqs):
    length = np.array([len(s) for s in seqs], np.uint32)
    off = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.uint64)
    return np.concatenate(seqs).astype(np.uint8), off, length


def test_reverse_strand_identical_closed_form():
    # B is the reverse complement of A: on the reverse strand the reads are
    # identical, so the best alignment is the whole read (score = length)
    rng = np.random.default_rng(3)
    A = rand_codes(rng, 700)
    codes, off, length = _reads(A, op.revcomp(A))
    for pa in (0, 250, 683):
        out = op.align_pairs(codes, off, length, [(0, 1)], [0, 1], [(pa, pa)], rc=[1], x_scalar=25)
        assert out["status"][0] == 0 and out["score"][0] == 700
        assert out["beg"][0].tolist() == [0, 0] and out["end"][0].tolist() == [700, 700]
        assert out["cells"][0] > 0 and out["seed_idx"][0] == 0 and out["n_kept"][0] == 1
    # forward, the same two reads are unrelated and the seed is not shared
    fwd = op.align_pairs(codes, off, length, [(0, 1)], [0, 1], [(250, 250)], rc=[0], x_scalar=25)
    assert fwd["score"][0] < 700


def test_best_of_seeds_and_tie_rule():
    rng = np.random.default_rng(5)
    A = rand_codes(rng, 3000)
    # B: A's bases 1000..1999 exact, flanked by unrelated sequence
    B = np.concatenate([rand_codes(rng, 500), A[1000:2000], rand_codes(rng, 500)])
    codes, off, length = _reads(A, B)
    # seed 0 is a spurious 17-mer match planted far from the overlap; seeds 1
    # and 2 lie on the true overlap and reach the same best score
    B2 = B.copy()
    B2[100:117] = A[2500:2517]
    codes, off, length = _reads(A, B2)
    seeds = [(1100, 600), (1500, 1000), (2500, 100)]
    order = np.argsort([s[0] for s in seeds])
    seeds = [seeds[i] for i in order]
    out = op.align_pairs(codes, off, length, [(0, 1)], [0, 3], seeds, x_scalar=25, min_dist=17)
    each = [oracle.align_task(codes, off, length, 0, 1, s[0], s[1], 25) for s in seeds]
    scores = [e["score"] for e in each]
    best = int(np.argmax(scores))          # argmax returns the first of equal maxima
    assert out["score"][0] == max(scores) and out["seed_idx"][0] == best
    assert out["cells"][0] == sum(e["cells"] for e in each)
    assert scores[0] == scores[1] and best == 0   # the tie goes to the earlier seed
    # max_seeds = 1 keeps the first seed only; min_dist 1000 drops the second
    one = op.align_pairs(codes, off, length, [(0, 1)], [0, 3], seeds, x_scalar=25, max_seeds=1)
    assert one["n_kept"][0] == 1 and one["score"][0] == scores[0]
    kb = op.align_pairs(codes, off, length, [(0, 1)], [0, 3], seeds, x_scalar=25, min_dist=1000)
    assert kb["n_kept"][0] == 2 and kb["seed_idx"][0] in (0, 2)


def test_empty_list_and_invalid_seed():
    rng = np.random.default_rng(7)
    A = rand_codes(rng, 400)
    B = A.copy()
    codes, off, length = _reads(A, B)
    out = op.align_pairs(codes, off, length, [(0, 1), (0, 1), (0, 1)], [0, 0, 2, 3],
                         [(5, 390), (100, 100), (5, 390)], x_scalar=7)
    assert out["status"][0] == op.TASK_NO_SEED and out["n_kept"][0] == 0
    assert out["score"][0] == np.iinfo(np.int32).min and out["seed_idx"][0] == op.NO_SEED_IDX
    # pair 1: the first seed runs past B's end (invalid), the second aligns
    assert out["status"][1] == 0 and out["seed_idx"][1] == 1 and out["n_kept"][1] == 2
    assert out["score"][1] == 400
    # pair 2: its only seed is invalid, so the pair reports that seed's status
    assert out["status"][2] == oracle.TASK_BAD_SEED and out["seed_idx"][2] == op.NO_SEED_IDX
