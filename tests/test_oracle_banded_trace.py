"""Pins for the banded traceback oracle (oracle/banded_oracle.c,
xo_banded_trace): a hand case that fixes the tie rule, and properties of the
alignment it returns on random pairs — the ops re-score to the best score,
consume exactly the begin..end ranges, stay inside the band, start and end on
matches — with best, end and cells equal to the untraced oracle's."""
import numpy as np

import oracle

M, I, D = oracle.OP_M, oracle.OP_I, oracle.OP_D


def cigar(ops):
    return "".join("%d%s" % (int(e) >> 2, "MID"[int(e) & 3]) for e in ops)


def test_hand_case_tie_rule():
    # A = ACGTTACG, B = ACGTACG: one of A's two T's is unmatched, score 7 - 1.
    # Walking back from (8, 7), cell (5, 4) is reached both diagonally from
    # H(4, 3) = 2 and from above, H(4, 4) = 4 plus a gap: the diagonal wins, so
    # the gap is A's first T: 3M 1D 4M (preferring "up" would give 4M1D3M).
    best, i, j, cells, bi, bj, ops = oracle.banded_trace("ACGTTACG", "ACGTACG", 0, 3)
    assert (best, i, j, bi, bj) == (6, 8, 7, 0, 0)
    assert cigar(ops) == "3M1D4M"
    # B gains the T instead: the gap moves to B (an I step).  Walking back from
    # (7, 8), cell (4, 5) holds 3 both from the diagonal, H(3, 4) = 2 plus the
    # T/T match, and from the left, H(4, 4) = 4 plus a gap: the diagonal wins,
    # so the gap is B's first T (3M 1I 4M; preferring "left" gives 4M1I3M).
    best, i, j, cells, bi, bj, ops = oracle.banded_trace("ACGTACG", "ACGTTACG", 0, 3)
    assert (best, i, j, bi, bj) == (6, 7, 8, 0, 0)
    assert cigar(ops) == "3M1I4M"
    # local: a mismatching prefix and suffix are cut away
    best, i, j, cells, bi, bj, ops = oracle.banded_trace("TTACGTAA", "GGACGTCC", 0, 2)
    assert (best, bi, bj, i, j) == (4, 2, 2, 6, 6) and cigar(ops) == "4M"
    # nothing positive: empty alignment at (0, 0)
    best, i, j, cells, bi, bj, ops = oracle.banded_trace("AAAA", "CCCC", 0, 1)
    assert (best, i, j, bi, bj, ops.size) == (0, 0, 0, 0, 0, 0)


def test_hand_case_up_before_left():
    # Scores +1/-3/-1: the A/C substitution in the middle costs more than a gap
    # on each side (-3 < -2).  A = ACGTAGGGG, B = ACGTCGGGG, band w = 4 around
    # the main diagonal.  The best local score is 6 (eight matches, two gaps),
    # ending at (9, 9).  Walking back, the four G
    # matches lead to (5, 5), H = 2, where the diagonal gives H(4, 4) - 3 = 1
    # while (i-1, j) and (i, j-1) both give 3 - 1 = 2 (H(4, 5) = H(5, 4) = 3).
    # Preferring (i-1, j) takes A's base against a gap (D) first when walking
    # back, then B's C (I) from (4, 5): forwards 4M 1I 1D 4M.  Preferring
    # (i, j-1) would give 4M1D1I4M.
    best, i, j, cells, bi, bj, ops = oracle.banded_trace("ACGTAGGGG", "ACGTCGGGG", 0, 4,
                                                         1, -3, -1)
    assert (best, i, j, bi, bj) == (6, 9, 9, 0, 0)
    assert cigar(ops) == "4M1I1D4M"


def check_alignment(a, b, c, w, got, match=1, mismatch=-1, gap=-1):
    best, i, j, cells, bi, bj, ops = got
    assert (best, i, j, cells) == oracle.banded(a, b, c, w, match, mismatch, gap)
    if best == 0:
        assert (bi, bj, ops.size) == (0, 0, 0)
        return
    x, y, score = bi, bj, 0
    cols = []
    for e in ops:
        n, op = int(e) >> 2, int(e) & 3
        assert n >= 1 and op in (M, I, D)
        for _ in range(n):
            if op == M:
                x, y = x + 1, y + 1
                score += match if a[x - 1] == b[y - 1] else mismatch
            elif op == D:
                x += 1
                score += gap
            else:
                y += 1
                score += gap
            assert abs(x - y - c) <= w, "path leaves the band"
            cols.append(op)
    assert (x, y) == (i, j), "ops do not end at the end cell"
    assert score == best, "ops re-score to %d, not %d" % (score, best)
    assert cols[0] == M and a[bi] == b[bj], "alignment does not start on a match"
    assert cols[-1] == M and a[i - 1] == b[j - 1], "alignment does not end on a match"
    # run-length entries alternate ops
    assert all((int(p) & 3) != (int(q) & 3) for p, q in zip(ops[:-1], ops[1:]))


def test_random_pairs_properties():
    rng = np.random.default_rng(17)
    for t in range(300):
        n = int(rng.integers(0, 300))
        a = rng.integers(0, 4, n).astype(np.uint8)
        # b = a with about 8 % deletions, 8 % insertions, 8 % substitutions
        out = []
        for u, r in enumerate(rng.random(n)):
            if r < 0.08:
                continue                                   # deleted
            if r < 0.16:
                out.append(int(rng.integers(0, 4)))        # inserted before a[u]
            out.append(int(rng.integers(0, 4)) if r > 0.92 else int(a[u]))
        b = np.array(out, np.uint8)
        if t % 5 == 0:
            b = rng.integers(0, 4, int(rng.integers(0, 200))).astype(np.uint8)
        w = int(rng.integers(0, 49))
        c = int(rng.integers(-20, 21))
        sc = [(1, -1, -1), (2, -3, -2), (1, -2, -1)][t % 3]
        got = oracle.banded_trace(a, b, c, w, *sc)
        check_alignment(a, b, c, w, got, *sc)
