"""Pins for the CPU oracle (no GPU).

Every check compares the oracle with something it does not share code with:
hand-worked vectors, exhaustive enumeration of alignments (section 2
definition), the textbook full dynamic programme (X = infinity), a full-grid
brute force of the X-drop rule, closed forms for identical and contained
reads, and invariants.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = json.load(open(os.path.join(HERE, "golden", "hand_vectors.json")))
ACGT = "ACGT"


def rand_seq(rng, n, alphabet=ACGT):
    return "".join(rng.choice(list(alphabet), n)) if n else ""


def mutate(rng, s, p=0.15):
    out = []
    for c in s:
        r = rng.random()
        if r < p / 3:
            continue                              # deletion
        if r < 2 * p / 3:
            out.append(rng.choice([x for x in ACGT if x != c]))  # substitution
        else:
            out.append(c)
        if rng.random() < p / 3:
            out.append(rng.choice(list(ACGT)))    # insertion
    return "".join(out)


@pytest.mark.parametrize("vec", GOLDEN["extensions"], ids=lambda v: v["id"])
def test_hand_vectors(vec):
    got = oracle.extend(vec["a"], vec["b"], vec["X"])
    assert got == (vec["best"], vec["i"], vec["j"], vec["cells"])


def test_hand_vectors_brute_agrees():
    # the full-grid brute force must reproduce the same hand computation
    for vec in GOLDEN["extensions"]:
        assert brute.xdrop_grid(vec["a"], vec["b"], vec["X"]) == (
            vec["best"], vec["i"], vec["j"], vec["cells"]), vec["id"]


def test_enumeration_small_alphabet_exhaustive():
    # every string pair over {A,C} up to length 4: X = inf equals the best of
    # all alignments of all prefix pairs; every cell but the origin evaluated
    for la in range(0, 5):
        for lb in range(0, 5):
            for a in itertools.product("AC", repeat=la):
                for b in itertools.product("AC", repeat=lb):
                    a_, b_ = "".join(a), "".join(b)
                    best, i, j, cells = oracle.extend(a_, b_, oracle.X_INF)
                    assert best == brute.enumerate_best(a_, b_), (a_, b_)
                    assert cells == (la + 1) * (lb + 1) - 1


def test_enumeration_random_len6():
    rng = np.random.default_rng(1)
    for _ in range(60):
        a = rand_seq(rng, int(rng.integers(0, 7)))
        b = rand_seq(rng, int(rng.integers(0, 7)))
        for (M, MM, G) in ((1, -1, -1), (2, -3, -2), (1, -2, -1)):
            best = oracle.extend(a, b, oracle.X_INF, M, MM, G)[0]
            assert best == brute.enumerate_best(a, b, M, MM, G), (a, b, M, MM, G)


@pytest.mark.parametrize("scoring", [(1, -1, -1), (2, -3, -2), (5, -4, -3), (1, -1, -2)])
def test_infinite_x_equals_full_dp(scoring):
    M, MM, G = scoring
    rng = np.random.default_rng(2)
    for t in range(40):
        la, lb = int(rng.integers(0, 60)), int(rng.integers(0, 60))
        a = rand_seq(rng, la)
        b = mutate(rng, a)[:lb] if t % 2 else rand_seq(rng, lb)
        best, i, j, cells = oracle.extend(a, b, oracle.X_INF, M, MM, G)
        assert (best, i, j) == brute.full_dp(a, b, M, MM, G), (a, b)
        assert cells == (len(a) + 1) * (len(b) + 1) - 1


@pytest.mark.parametrize("scoring", [(1, -1, -1), (2, -3, -2), (1, -2, -1)])
def test_xdrop_equals_grid_bruteforce(scoring):
    M, MM, G = scoring
    rng = np.random.default_rng(3)
    for t in range(150):
        la = int(rng.integers(0, 40))
        alpha = "AC" if t % 3 == 0 else ACGT  # small alphabets create ties
        a = rand_seq(rng, la, alpha)
        b = mutate(rng, a, 0.3) if t % 2 else rand_seq(rng, int(rng.integers(0, 40)), alpha)
        X = int(rng.integers(0, 12))
        assert oracle.extend(a, b, X, M, MM, G) == brute.xdrop_grid(a, b, X, M, MM, G), (a, b, X)


def test_identical_sequences_closed_form():
    rng = np.random.default_rng(4)
    for L in (1, 7, 50, 333):
        a = rand_seq(rng, L)
        for X in (0, 1, 5, 40):
            best, i, j, _ = oracle.extend(a, a, X)
            assert (best, i, j) == (L, L, L)


def test_prefix_containment_closed_form():
    # b is a prefix of a: the best extension consumes all of b on the diagonal
    rng = np.random.default_rng(5)
    a = rand_seq(rng, 200)
    for lb in (0, 1, 60, 199):
        b = a[:lb]
        for X in (0, 3, 25):
            assert oracle.extend(a, b, X)[:3] == (lb, lb, lb)


def test_invariants_random():
    rng = np.random.default_rng(6)
    for _ in range(80):
        a = rand_seq(rng, int(rng.integers(0, 120)))
        b = mutate(rng, a, 0.2)
        X = int(rng.integers(0, 30))
        best, i, j, cells = oracle.extend(a, b, X)
        best_inf = oracle.extend(a, b, oracle.X_INF)[0]
        assert 0 <= best <= best_inf
        assert 0 <= i <= len(a) and 0 <= j <= len(b)
        # swapping the sequences transposes the grid: same best and cell count
        sb, si, sj, sc = oracle.extend(b, a, X)
        assert (sb, sc) == (best, cells)
        assert cells <= (len(a) + 1) * (len(b) + 1) - 1


def _task_arrays(reads):
    codes = np.concatenate([np.array(["ACGT".index(c) for c in r], np.uint8) for r in reads])
    length = np.array([len(r) for r in reads], np.uint32)
    off = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.uint64)
    return codes, off, length


def test_task_identical_reads():
    rng = np.random.default_rng(7)
    A = rand_seq(rng, 100)
    codes, off, length = _task_arrays([A, A])
    r = oracle.align_task(codes, off, length, 0, 1, 40, 40, 25)
    assert r["status"] == oracle.TASK_OK
    assert r["score"] == 100 and r["beg"] == (0, 0) and r["end"] == (100, 100)


def test_task_containment():
    rng = np.random.default_rng(8)
    A = rand_seq(rng, 150)
    B = A[30:]
    codes, off, length = _task_arrays([A, B])
    r = oracle.align_task(codes, off, length, 0, 1, 50, 20, 25)
    assert r["score"] == len(B)
    assert r["beg"] == (30, 0) and r["end"] == (150, len(B))


def test_task_seed_is_ungapped_sum():
    # seed at the very start and end of both reads: no extension possible
    codes, off, length = _task_arrays(["ACGTACGTACGTACGTA", "ACGTACGTACGTACGTT"])
    r = oracle.align_task(codes, off, length, 0, 1, 0, 0, 10)
    assert r["score"] == 16 - 1 and r["cells"] == 0
    assert r["beg"] == (0, 0) and r["end"] == (17, 17)


def test_task_status_codes():
    codes, off, length = _task_arrays(["ACGTACGTACGTACGTACGT", "ACGTACGTACGTACGTACGT"])
    assert oracle.align_task(codes, off, length, 0, 2, 0, 0, 5)["status"] == oracle.TASK_BAD_READ
    assert oracle.align_task(codes, off, length, 0, 1, 4, 0, 5)["status"] == oracle.TASK_BAD_SEED
    assert oracle.align_task(codes, off, length, 0, 1, 0, 4, 5)["status"] == oracle.TASK_BAD_SEED
    r = oracle.align_task(codes, off, length, 0, 1, 3, 3, 5)
    assert r["status"] == oracle.TASK_OK
    assert oracle.align_task(codes, off, length, 0, 1, 0, 0, -1)["status"] == oracle.TASK_BAD_X
    bad = oracle.align_task(codes, off, length, 0, 1, 0, 0, oracle.X_MAX + 1)
    assert bad["status"] == oracle.TASK_BAD_X and bad["score"] == -2**31 and bad["cells"] == 0


def test_param_checks():
    assert oracle.check_params(17, 1, -1, -1)
    assert not oracle.check_params(0, 1, -1, -1)
    assert not oracle.check_params(17, 0, -1, -1)
    assert not oracle.check_params(17, 1, 1, -1)
    assert not oracle.check_params(17, 1, -1, 0)


def test_batch_matches_single_tasks():
    import synth
    w = synth.config("c1-small")
    res = oracle.align_workload(w, n_threads=4)
    for t in range(0, w.n_tasks, 7):
        r = oracle.align_task(w.codes, w.off, w.length, int(w.ra[t]), int(w.rb[t]),
                              int(w.pa[t]), int(w.pb[t]), int(w.x[t]))
        assert r["score"] == res["score"][t]
        assert r["beg"] == tuple(res["beg"][t]) and r["end"] == tuple(res["end"][t])
        assert r["cells"] == res["cells"][t]


def test_workload_tasks_are_true_overlaps():
    # the generator's seeds are exact shared k-mers, so every task scores at
    # least k and its alignment contains the seed
    import synth
    w = synth.config("c1-small")
    res = oracle.align_workload(w, n_threads=4)
    assert (res["status"] == 0).all()
    assert (res["score"] >= w.k).all()
    assert (res["beg"][:, 0] <= w.pa).all() and (res["end"][:, 0] >= w.pa + w.k).all()
