"""Pins for the banded Smith-Waterman oracle (oracle/banded_oracle.c):
exhaustive path enumeration on tiny inputs, the unbanded case against local
alignment built from the pinned anchored dynamic programme, closed forms for
identical sequences and for a zero-width band, the band's cell count."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute

from helpers import mutate_codes, rand_codes

SCHEMES = [(1, -1, -1), (2, -3, -2), (1, -1, -3)]


def _in_band(i, j, c, w):
    return abs(i - j - c) <= w


def _paths_brute(a, b, c, w, M, MM, G):
    """H(i, j) = max(0, best score of a path of moves ending at (i, j)), by
    enumerating every path: it starts at a boundary point (row or column 0)
    or an in-band cell with score 0 and steps diagonally (scoring the pair it
    lands on) or by a gap, landing only on in-band cells."""
    m, n = len(a), len(b)
    H = {}
    starts = [(i, j) for i in range(m + 1) for j in range(n + 1)
              if i == 0 or j == 0 or _in_band(i, j, c, w)]

    def walk(i, j, score):
        for di, dj in ((1, 1), (1, 0), (0, 1)):
            u, v = i + di, j + dj
            if u > m or v > n or not _in_band(u, v, c, w):
                continue
            s = score + ((M if a[u - 1] == b[v - 1] else MM) if di and dj else G)
            H[(u, v)] = max(H.get((u, v), 0), s)
            walk(u, v, s)

    for i, j in starts:
        walk(i, j, 0)
    best, bi, bj = 0, 0, 0
    for d in range(2, m + n + 1):
        for i in range(max(1, d - n), min(m, d - 1) + 1):
            h = H.get((i, d - i), 0 if _in_band(i, d - i, c, w) else None)
            if h is not None and h > best:
                best, bi, bj = h, i, d - i
    cells = sum(1 for i in range(1, m + 1) for j in range(1, n + 1) if _in_band(i, j, c, w))
    return best, bi, bj, cells


@pytest.mark.parametrize("scheme", SCHEMES)
def test_tiny_exhaustive(scheme):
    rng = np.random.default_rng(sum(scheme) + 9)
    for _ in range(40):
        m, n = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        a = rng.integers(0, 2, m).tolist()   # two letters: many ties
        b = rng.integers(0, 2, n).tolist()
        c, w = int(rng.integers(-3, 4)), int(rng.integers(0, 3))
        assert oracle.banded(a, b, c, w, *scheme) == _paths_brute(a, b, c, w, *scheme), (a, b, c, w)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_unbanded_equals_local_alignment(scheme):
    # a band wider than the grid is plain Smith-Waterman: the best over all
    # start points (i0, j0) of the anchored, free-end optimum of the suffixes
    rng = np.random.default_rng(sum(scheme) + 17)
    for _ in range(25):
        m, n = int(rng.integers(0, 25)), int(rng.integers(0, 25))
        a = rng.integers(0, 4, m).tolist()
        b = rng.integers(0, 4, n).tolist()
        best = 0
        for i0, j0 in itertools.product(range(m + 1), range(n + 1)):
            best = max(best, brute.full_dp(a[i0:], b[j0:], *scheme)[0])
        got = oracle.banded(a, b, 0, m + n, *scheme)
        assert got[0] == best and got[3] == m * n


def test_identical_and_zero_width():
    rng = np.random.default_rng(2)
    a = rand_codes(rng, 300)
    for w in (0, 5, 31, 48):
        best, i, j, _ = oracle.banded(a, a, 0, w)
        assert (best, i, j) == (300, 300, 300)
    # w = 0: only the diagonal i - j = c; the best is the largest sum of a run
    # of consecutive +1/-1 match scores along it (Kadane), first reached
    b = mutate_codes(rng, a, 0.3)
    for c in (-7, 0, 4):
        diag = [1 if a[i - 1] == b[i - c - 1] else -1
                for i in range(max(1, 1 + c), min(len(a), len(b) + c) + 1)]
        best = run = 0
        for s in diag:
            run = max(0, run + s)
            best = max(best, run)
        assert oracle.banded(a, b, c, 0)[0] == best


def test_band_cell_count_closed_form():
    rng = np.random.default_rng(4)
    for _ in range(30):
        m, n = int(rng.integers(0, 200)), int(rng.integers(0, 200))
        c, w = int(rng.integers(-250, 250)), int(rng.integers(0, 49))
        # one diagonal delta = i - j per band offset: its length inside the grid
        expect = sum(max(0, min(m, n + dlt) - max(1, 1 + dlt) + 1)
                     for dlt in range(c - w, c + w + 1))
        a, b = rand_codes(rng, m), rand_codes(rng, n)
        assert oracle.banded(a, b, c, w)[3] == expect


def test_task_statuses():
    rng = np.random.default_rng(6)
    A = rand_codes(rng, 500)
    codes, off, length = A, np.array([0], np.uint64), np.array([500], np.uint32)
    r = oracle.banded_batch(codes, off, length, [(0, 0), (0, 1), (0, 0), (0, 0)],
                            [(10, 10), (0, 0), (490, 0), (10, 10)], w=[8, 8, 8, 49])
    assert r["status"].tolist() == [0, oracle.TASK_BAD_READ, oracle.TASK_BAD_SEED,
                                    oracle.TASK_BAD_X]
    assert r["score"][0] == 500 and r["end"][0].tolist() == [500, 500]
