"""Pins for the candidate-pair oracle (oracle/overlap.py): brute-force
substring comparison on small read sets, a hand case, the count filter."""
import numpy as np

from oracle import overlap as ov

from helpers import rand_codes


def _reads(*seqs):
    length = np.array([len(s) for s in seqs], np.uint32)
    off = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.uint64)
    return np.concatenate(seqs).astype(np.uint8), off, length


def test_hand_case():
    # k = 3; read 0 = AAAC, read 1 = CAAAC, read 2 = GGGG
    codes, off, length = _reads([0, 0, 0, 1], [1, 0, 0, 0, 1], [2, 2, 2, 2])
    pairs, so, seeds, st = ov.find_overlaps(codes, off, length, k=3, count_lo=2, count_hi=8)
    # AAA: (0,0) (1,1); AAC: (0,1) (1,2); CAA only in read 1; GGG twice in read 2
    assert pairs.tolist() == [[0, 1]]
    assert seeds.tolist() == [[0, 1], [1, 2]] and so.tolist() == [0, 2]
    assert st == dict(kmers=2 + 3 + 2, distinct=4, retained=3, occurrences=6,
                    non_singletons=3)
    # GGG occurs twice but only within read 2: retained, yet no pair; with
    # count_hi = 1 nothing is retained
    assert ov.find_overlaps(codes, off, length, 3, 2, 1)[0].size == 0


def test_brute_force_small_sets():
    rng = np.random.default_rng(3)
    for trial in range(12):
        n_reads = int(rng.integers(2, 7))
        k = int(rng.integers(2, 6))
        lo, hi = 2, int(rng.integers(2, 9))
        seqs = [rng.integers(0, 3 if trial % 2 else 4, int(rng.integers(0, 40))).astype(np.uint8)
                for _ in range(n_reads)]
        codes, off, length = _reads(*seqs) if seqs else _reads(np.zeros(0, np.uint8))
        pairs, so, seeds, _ = ov.find_overlaps(codes, off, length, k, lo, hi)
        got = {(int(a), int(b)): [tuple(int(v) for v in s) for s in seeds[int(so[i]):int(so[i + 1])]]
               for i, (a, b) in enumerate(pairs)}
        # brute force: count every substring of length k, then compare all
        # position pairs of different reads directly
        def sub(r, p):
            return tuple(seqs[r][p:p + k].tolist())
        count = {}
        for r, s in enumerate(seqs):
            for p in range(len(s) - k + 1):
                count[sub(r, p)] = count.get(sub(r, p), 0) + 1
        expect = {}
        for ra in range(n_reads):
            for rb in range(ra + 1, n_reads):
                for pa in range(len(seqs[ra]) - k + 1):
                    for pb in range(len(seqs[rb]) - k + 1):
                        if sub(ra, pa) == sub(rb, pb) and lo <= count[sub(ra, pa)] <= hi:
                            expect.setdefault((ra, rb), []).append((pa, pb))
        assert got == {key: sorted(v) for key, v in expect.items()}, trial


def test_planted_overlap():
    rng = np.random.default_rng(5)
    A, B = rand_codes(rng, 2000), rand_codes(rng, 2000)
    B[500:1500] = A[1000:2000]   # exact 1 kbp overlap at shift 500
    codes, off, length = _reads(A, B)
    pairs, so, seeds, st = ov.find_overlaps(codes, off, length, 17, 2, 8)
    assert pairs.tolist() == [[0, 1]]
    # every 17-mer of the shared 1 kbp is a seed on the shift-500 diagonal;
    # a few more may join where B's random flank happens to continue the copy
    diag = {pb for pa, pb in seeds.tolist() if pa - pb == 500}
    assert set(range(500, 1500 - 17 + 1)) <= diag
    for pa, pb in seeds.tolist():
        assert np.array_equal(A[pa:pa + 17], B[pb:pb + 17])


def test_sorted_variant_matches():
    # the sort-based form (for large read sets) equals the dict form,
    # statistics included, with repeats, short reads and several bounds
    rng = np.random.default_rng(9)
    for trial in range(10):
        base = rand_codes(rng, 3000)
        seqs = []
        for _ in range(int(rng.integers(1, 30))):
            n = int(rng.integers(0, 400))
            s = int(rng.integers(0, 3000 - n + 1))
            r = base[s:s + n].copy()
            flip = rng.random(n) < 0.05
            r[flip] = rng.integers(0, 4, int(flip.sum()))
            seqs.append(r.astype(np.uint8))
        if trial % 3 == 0:
            seqs.append(np.zeros(100, np.uint8))          # homopolymer: one k-mer, many times
        codes, off, length = _reads(*seqs)
        k = int(rng.choice([5, 11, 17, 31]))
        lo, hi = 2, int(rng.integers(1, 12))
        a = ov.find_overlaps(codes, off, length, k, lo, hi)
        b = ov.find_overlaps_sorted(codes, off, length, k, lo, hi)
        for x, y in zip(a[:3], b[:3]):
            assert x.dtype == y.dtype and np.array_equal(x, y), trial
        assert a[3] == b[3], trial
