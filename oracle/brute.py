"""Tiny brute-force checks for the oracle: TEST INFRASTRUCTURE ONLY.

Three independent routes to results the X-drop extension must reproduce:

* `enumerate_best`: every alignment (section 2 definition: equal-length gapped
  strings, no all-gap column, deleting gaps gives the inputs) of every prefix
  pair a[1..i], b[1..j], scored column by column.  With no pruning (X large)
  the extension's best must equal the maximum over all of them.
* `full_dp`: the textbook dynamic programme over the whole (m+1) x (n+1)
  table with the start anchored at (0,0) and a free end, as in exact
  Smith-Waterman/Needleman-Wunsch (section 2).  Same role, any size.
* `xdrop_grid`: the X-drop rule applied to every cell of every antidiagonal
  of the full table, with no row-range bookkeeping and no early stop.  It
  checks the oracle's range restriction and stopping rule on small inputs.

Pure Python; only for inputs of a few dozen characters.
"""
from __future__ import annotations

NEG = None  # marks a dead / unreachable cell


def _codes(s):
    if isinstance(s, str):
        return [{"A": 0, "C": 1, "G": 2, "T": 3}[c] for c in s]
    return [int(v) for v in s]


def enumerate_best(a, b, match=1, mismatch=-1, gap=-1):
    """Max score over all alignments of all prefix pairs (incl. the empty one).

    Alignments are walked as column sequences: each column consumes one
    character of a, one of b, or both (never neither).
    """
    a, b = _codes(a), _codes(b)
    m, n = len(a), len(b)
    best = [0]

    def walk(i, j, score):
        # (i, j): characters consumed; every prefix pair reached is a candidate
        if score > best[0]:
            best[0] = score
        if i < m and j < n:
            walk(i + 1, j + 1, score + (match if a[i] == b[j] else mismatch))
        if i < m:
            walk(i + 1, j, score + gap)
        if j < n:
            walk(i, j + 1, score + gap)

    walk(0, 0, 0)
    return best[0]


def full_dp(a, b, match=1, mismatch=-1, gap=-1):
    """Anchored-start, free-end optimum -> (best, i, j) with the arg-max taken
    at the smallest antidiagonal i+j, then the smallest i."""
    a, b = _codes(a), _codes(b)
    m, n = len(a), len(b)
    H = [[0] * (n + 1) for _ in range(m + 1)]
    for i in range(1, m + 1):
        H[i][0] = i * gap
    for j in range(1, n + 1):
        H[0][j] = j * gap
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            H[i][j] = max(H[i - 1][j - 1] + (match if a[i - 1] == b[j - 1] else mismatch),
                          H[i - 1][j] + gap, H[i][j - 1] + gap)
    best, bi, bj = 0, 0, 0
    for d in range(0, m + n + 1):
        for i in range(max(0, d - n), min(m, d) + 1):
            if H[i][d - i] > best:
                best, bi, bj = H[i][d - i], i, d - i
    return best, bi, bj


def xdrop_grid(a, b, X, match=1, mismatch=-1, gap=-1):
    """X-drop over the full grid -> (best, i, j, cells)."""
    a, b = _codes(a), _codes(b)
    m, n = len(a), len(b)
    S = [[NEG] * (n + 1) for _ in range(m + 1)]  # live scores only
    S[0][0] = 0
    T, bi, bj, cells = 0, 0, 0, 0
    for d in range(1, m + n + 1):
        t_prev = T
        row_best, row_i = None, None
        for i in range(0, m + 1):
            j = d - i
            if j < 0 or j > n:
                continue
            cand = []
            if i >= 1 and j >= 1 and S[i - 1][j - 1] is not NEG:
                cand.append(S[i - 1][j - 1] + (match if a[i - 1] == b[j - 1] else mismatch))
            if i >= 1 and S[i - 1][j] is not NEG:
                cand.append(S[i - 1][j] + gap)
            if j >= 1 and S[i][j - 1] is not NEG:
                cand.append(S[i][j - 1] + gap)
            if not cand:
                continue
            cells += 1
            s = max(cand)
            if s >= t_prev - X:
                S[i][j] = s
                if row_best is None or s > row_best:
                    row_best, row_i = s, i
        if row_best is not None and row_best > T:
            T, bi, bj = row_best, row_i, d - row_i
    return T, bi, bj, cells
