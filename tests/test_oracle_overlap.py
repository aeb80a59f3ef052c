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


# ---- both strands (canonical k-mers with a strand bit) ------------------------

def _revcomp(s):
    return (3 - np.asarray(s, np.uint8)[::-1]).astype(np.uint8)


def _as_dict(res):
    pairs, so, seeds, _, rc = res
    return {(int(a), int(b), int(r)): [tuple(int(v) for v in s)
                                       for s in seeds[int(so[i]):int(so[i + 1])]]
            for i, ((a, b), r) in enumerate(zip(pairs, rc))}


def test_revcomp_codes():
    # AACG (0,0,1,2) -> reverse complement CGTT (1,2,3,3)
    code = ov.kmer_codes(np.array([0, 0, 1, 2], np.uint8), 4)
    assert ov.revcomp_codes(code, 4).tolist() == ov.kmer_codes(np.array([1, 2, 3, 3]), 4).tolist()
    rng = np.random.default_rng(1)
    s = rand_codes(rng, 200)
    for k in (1, 5, 17, 32):
        f = ov.kmer_codes(s, k)
        assert np.array_equal(ov.revcomp_codes(ov.revcomp_codes(f, k), k), f)
        # the k-mer at p read on the other strand is the k-mer at n - k - p of
        # the reversed complement
        assert np.array_equal(ov.revcomp_codes(f, k), ov.kmer_codes(_revcomp(s), k)[::-1])


def test_both_strands_brute_force():
    rng = np.random.default_rng(4)
    for trial in range(14):
        n_reads = int(rng.integers(2, 7))
        k = int(rng.choice([1, 3, 5]))          # odd: no k-mer is its own reverse complement
        lo, hi = 2, int(rng.integers(2, 9))
        seqs = [rng.integers(0, 4, int(rng.integers(0, 30))).astype(np.uint8)
                for _ in range(n_reads)]
        codes, off, length = _reads(*seqs)
        got = _as_dict(ov.find_overlaps(codes, off, length, k, lo, hi, strands=2))

        def sub(r, p):
            return tuple(seqs[r][p:p + k].tolist())

        def rcs(t):
            return tuple(3 - v for v in reversed(t))

        def canon(t):
            return min(t, rcs(t))
        count = {}
        for r, s in enumerate(seqs):
            for p in range(len(s) - k + 1):
                count[canon(sub(r, p))] = count.get(canon(sub(r, p)), 0) + 1
        expect = {}
        for ra in range(n_reads):
            for rb in range(ra + 1, n_reads):
                lb = len(seqs[rb])
                for pa in range(len(seqs[ra]) - k + 1):
                    for pb in range(lb - k + 1):
                        a, b = sub(ra, pa), sub(rb, pb)
                        if not lo <= count[canon(a)] <= hi:
                            continue
                        if a == b:
                            expect.setdefault((ra, rb, 0), []).append((pa, pb))
                        if a == rcs(b):
                            expect.setdefault((ra, rb, 1), []).append((pa, lb - k - pb))
        assert got == {key: sorted(v) for key, v in expect.items()}, trial


def test_reverse_complement_twin():
    # a read and its reverse complement share every 17-mer on opposite
    # strands: one rc pair whose seeds are (p, p) in rb' coordinates
    rng = np.random.default_rng(6)
    R, U = rand_codes(rng, 500), rand_codes(rng, 400)
    codes, off, length = _reads(R, _revcomp(R), U)
    pairs, so, seeds, st, rc = ov.find_overlaps(codes, off, length, 17, 2, 8, strands=2)
    assert pairs.tolist() == [[0, 1]] and rc.tolist() == [1]
    assert seeds.tolist() == [[p, p] for p in range(500 - 17 + 1)]
    assert st["retained"] == 500 - 17 + 1
    # forward k-mers alone see nothing shared
    assert ov.find_overlaps(codes, off, length, 17, 2, 8)[0].size == 0


def test_flipping_a_read_flips_its_pairs():
    rng = np.random.default_rng(7)
    base = rand_codes(rng, 1500)
    seqs = [base[s:s + 400].copy() for s in (0, 200, 500, 900, 1000)]
    codes, off, length = _reads(*seqs)
    ref = _as_dict(ov.find_overlaps(codes, off, length, 11, 2, 8, strands=2))
    assert ref
    for b in range(len(seqs)):
        flipped = list(seqs)
        flipped[b] = _revcomp(seqs[b])
        codes2, off2, length2 = _reads(*flipped)
        got = _as_dict(ov.find_overlaps(codes2, off2, length2, 11, 2, 8, strands=2))
        # flipping rb: its k-mer at q becomes the one at |rb| - k - q on the
        # other strand, which is where a reverse-strand seed already counts
        # it, so the seeds stay and the strand flips; flipping ra moves both
        # coordinates (pb counts in the other strand of rb after the flip)
        expect = {}
        for (ra, rb, r), lst in ref.items():
            if rb == b:
                expect[(ra, rb, 1 - r)] = lst
            elif ra == b:
                la, lb = len(seqs[ra]), len(seqs[rb])
                expect[(ra, rb, 1 - r)] = sorted((la - 11 - pa, lb - 11 - pb) for pa, pb in lst)
            else:
                expect[(ra, rb, r)] = lst
        assert got == expect, b


def test_palindromic_kmers_pair_on_the_forward_strand_only():
    # k = 4: ACGT is its own reverse complement
    acgt = np.array([0, 1, 2, 3], np.uint8)
    codes, off, length = _reads(acgt, acgt)
    pairs, so, seeds, st, rc = ov.find_overlaps(codes, off, length, 4, 2, 8, strands=2)
    assert pairs.tolist() == [[0, 1]] and rc.tolist() == [0] and seeds.tolist() == [[0, 0]]


def test_sorted_variant_matches_both_strands():
    rng = np.random.default_rng(10)
    for trial in range(8):
        base = rand_codes(rng, 2000)
        seqs = []
        for _ in range(int(rng.integers(1, 25))):
            n = int(rng.integers(0, 300))
            s = int(rng.integers(0, 2000 - n + 1))
            r = base[s:s + n].copy()
            seqs.append(_revcomp(r) if rng.random() < 0.5 else r)
        codes, off, length = _reads(*seqs)
        k = int(rng.choice([4, 5, 11, 17]))
        lo, hi = 2, int(rng.integers(1, 12))
        a = ov.find_overlaps(codes, off, length, k, lo, hi, strands=2)
        b = ov.find_overlaps_sorted(codes, off, length, k, lo, hi, strands=2)
        for x, y in zip(a[:3] + a[4:], b[:3] + b[4:]):
            assert x.dtype == y.dtype and np.array_equal(x, y), trial
        assert a[3] == b[3], trial
