"""Candidate pairs on the GPU (xd_find_overlaps) against the oracle: small
read sets element by element over k, m and filter sizes; the c2-small read
set exactly; the full c2 read set (138 Mbp) by the digest of the oracle's
whole result recorded by tests/golden/make_overlap_digests.py."""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import overlap as ov
from oracle import pairs as opairs

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from digest import overlap_digest, reads_digest  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402

RECORD = json.load(open(os.path.join(HERE, "golden", "overlap_digests.json")))
EXACT = ("kmers", "non_singletons", "retained", "occurrences")


def _reads(seqs):
    length = np.array([len(s) for s in seqs], np.uint32)
    off = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.uint64) if seqs else \
        np.zeros(0, np.uint64)
    codes = np.concatenate(seqs).astype(np.uint8) if seqs else np.zeros(0, np.uint8)
    return codes, off, length


def gpu(codes, off, length, k, m, bloom_bits=0, capacity=None):
    with xd.ReadStore(codes, off, length) as st:
        r = xd.find_overlaps(st, k=k, m=m, bloom_bits=bloom_bits, capacity=capacity)
    torch.cuda.synchronize()
    return (r["pairs"].cpu().numpy().view(np.uint32).reshape(-1, 2),
            r["seed_off"].cpu().numpy().view(np.uint64),
            r["seeds"].cpu().numpy().view(np.uint32).reshape(-1, 2), r["counts"])


def assert_same(got, ref, label):
    for name, g, o in zip(("pairs", "seed_off", "seeds"), got[:3], ref[:3]):
        assert g.shape == o.shape and np.array_equal(g, o), "%s: %s differ" % (label, name)
    for f in EXACT:
        assert got[3][f] == ref[3][f], "%s: %s %d != %d" % (label, f, got[3][f], ref[3][f])
    assert got[3]["pairs"] == ref[0].shape[0] and got[3]["seeds"] == ref[2].shape[0]


def test_small_sets_match_oracle():
    rng = np.random.default_rng(21)
    for trial in range(40):
        base = rng.integers(0, 4, 4000).astype(np.uint8)
        seqs = []
        for _ in range(int(rng.integers(1, 40))):
            n = int(rng.integers(0, 700))
            s = int(rng.integers(0, 4000 - n + 1))
            r = base[s:s + n].copy()
            flip = rng.random(n) < 0.04
            r[flip] = rng.integers(0, 4, int(flip.sum()))
            seqs.append(r)
        if trial % 4 == 0:
            seqs.append(np.full(300, 2, np.uint8))   # one k-mer, far above m
        if trial % 5 == 1:
            seqs.append(np.tile(np.array([0, 1], np.uint8), 50))
        k = int(rng.choice([1, 2, 5, 11, 17, 31]))
        m = int(rng.choice([1, 2, 3, 8, 64]))
        codes, off, length = _reads(seqs)
        ref = ov.find_overlaps(codes, off, length, k, 2, m)
        got = gpu(codes, off, length, k, m)
        assert_same(got, ref, "trial %d (k=%d, m=%d, %d reads)" % (trial, k, m, len(seqs)))


def test_degenerate_inputs():
    for seqs in ([], [np.zeros(0, np.uint8)], [np.arange(10, dtype=np.uint8) % 4] * 3,
                 [np.zeros(16, np.uint8), np.zeros(16, np.uint8)]):
        codes, off, length = _reads(seqs)
        ref = ov.find_overlaps(codes, off, length, 17, 2, 8)
        got = gpu(codes, off, length, 17, 8)
        assert_same(got, ref, "%d reads" % len(seqs))
        assert got[1].tolist() == ref[1].tolist()


def test_c2_small_exact_and_filter_sizes():
    w = synth.config("c2-small")
    ref = ov.find_overlaps_sorted(w.codes, w.off, w.length, 17, 2, 8)
    rec = RECORD["c2-small"]
    assert reads_digest(w) == rec["reads"]
    assert overlap_digest(*ref[:3]) == rec["digest"]
    for bits in (4, 16, 64):  # the first filter's size changes speed, not the result
        got = gpu(w.codes, w.off, w.length, 17, 8, bloom_bits=bits)
        assert_same(got, ref, "c2-small bloom_bits=%d" % bits)


def test_table_regrowth():
    # a first table far too small fills up; it is doubled and the pass rerun
    # (about seven times here) without changing the result
    w = synth.config("c2-small")
    ref = gpu(w.codes, w.off, w.length, 17, 8)
    with xd.ReadStore.from_workload(w) as st:
        r = xd.find_overlaps(st, k=17, m=8, table_slots=4096)
        torch.cuda.synchronize()
        got = (r["pairs"].cpu().numpy().view(np.uint32).reshape(-1, 2),
               r["seed_off"].cpu().numpy().view(np.uint64),
               r["seeds"].cpu().numpy().view(np.uint32).reshape(-1, 2), r["counts"])
    assert got[3]["table_slots"] > 4 * 4096 and got[3]["table_keys"] > 4096
    for a, b in zip(got[:3], ref[:3]):
        assert np.array_equal(a, b)
    for f in EXACT + ("pairs", "seeds"):
        assert got[3][f] == ref[3][f]


def test_capacity_and_eagain():
    w = synth.config("c2-small")
    with xd.ReadStore.from_workload(w) as st:
        r = xd.find_overlaps(st, k=17, m=8)
        P, S = r["counts"]["pairs"], r["counts"]["seeds"]
        with pytest.raises(xd.XdropError) as e:
            xd.find_overlaps(st, k=17, m=8, capacity=(P - 1, S))
        assert e.value.code == xd._lib.XD_EAGAIN
        with pytest.raises(xd.XdropError):
            xd.find_overlaps(st, k=32, m=8)
        with pytest.raises(xd.XdropError):
            xd.find_overlaps(st, k=17, m=65)
        again = xd.find_overlaps(st, k=17, m=8, capacity=(P, S))
        for f in ("pairs", "seed_off", "seeds"):
            assert torch.equal(r[f], again[f])


def test_c2_full_read_set_matches_record():
    w = synth.config("c2")
    rec = RECORD["c2"]
    assert reads_digest(w) == rec["reads"]
    got = gpu(w.codes, w.off, w.length, rec["k"], rec["m"])
    for f in EXACT + ("pairs", "seeds"):
        assert got[3][f] == rec[f], "c2: %s %d != %d" % (f, got[3][f], rec[f])
    assert overlap_digest(*got[:3]) == rec["digest"]


def test_pairs_feed_alignment():
    # the candidate lists go straight into xd_align_pairs (one seed and all
    # seeds k apart); a sample of pairs is checked against the oracle
    w = synth.config("c2-small")
    with xd.ReadStore.from_workload(w) as st:
        r = xd.find_overlaps(st, k=17, m=8)
        P = r["counts"]["pairs"]
        idx = np.linspace(0, P - 1, 40).astype(np.int64)
        so = r["seed_off"].cpu().numpy()
        pairs_h = r["pairs"].cpu().numpy()
        seeds_h = r["seeds"].cpu().numpy()
        for max_seeds, min_dist in ((1, 17), (0, 17)):
            out = xd.align_pairs(st, r["pairs"], r["seed_off"], r["seeds"], x_scalar=25,
                                 min_dist=min_dist, max_seeds=max_seeds, k=17)
            torch.cuda.synchronize()
            sub_off = np.concatenate([[0], np.cumsum(so[idx + 1] - so[idx])]).astype(np.uint64)
            sub_seeds = np.concatenate([seeds_h[so[i]:so[i + 1]] for i in idx])
            ref = opairs.align_pairs(w.codes, w.off, w.length, pairs_h[idx], sub_off, sub_seeds,
                                     x_scalar=25, min_dist=min_dist, max_seeds=max_seeds, k=17)
            for f in ("score", "status", "seed_idx", "n_kept"):
                assert np.array_equal(out[f].cpu().numpy()[idx], ref[f]), (max_seeds, f)
            assert np.array_equal(out["cells"].cpu().numpy()[idx].astype(np.uint64),
                                  ref["cells"].astype(np.uint64))


def test_release_memory_between_calls():
    # scratch stays cached in the library's pool between calls; handing it
    # back changes nothing for the next call
    w = synth.config("c2-small")
    first = gpu(w.codes, w.off, w.length, 17, 8)
    xd.release_memory()
    again = gpu(w.codes, w.off, w.length, 17, 8)
    for a, b in zip(first[:3], again[:3]):
        assert np.array_equal(a, b)


def test_c2_candidates_align_like_the_oracle():
    # the pipeline at full size, as bench_overlap.py runs it: every candidate
    # pair of the c2 read set aligned from its first seed (chance pairs
    # included, whose extensions reach the wide windows); a sample of pairs,
    # half of them single-seed pairs (mostly chance collisions), against the
    # pair oracle
    w = synth.config("c2")
    with xd.ReadStore.from_workload(w) as st:
        r = xd.find_overlaps(st, k=17, m=8)
        out = xd.align_pairs(st, r["pairs"], r["seed_off"], r["seeds"], x_scalar=25,
                             min_dist=17, max_seeds=1, k=17, n_seeds=r["counts"]["seeds"])
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        so = r["seed_off"].cpu().numpy()
        pairs_h = r["pairs"].cpu().numpy()
        seeds_h = r["seeds"].cpu().numpy()
    assert (got["status"] == 0).all()
    rng = np.random.default_rng(4)
    single = np.nonzero(so[1:] - so[:-1] == 1)[0]
    idx = np.concatenate([rng.choice(single, 15, replace=False),
                          rng.choice(pairs_h.shape[0], 15, replace=False)])
    sub_off = np.concatenate([[0], np.cumsum(so[idx + 1] - so[idx])]).astype(np.uint64)
    sub_seeds = np.concatenate([seeds_h[so[i]:so[i + 1]] for i in idx])
    ref = opairs.align_pairs(w.codes, w.off, w.length, pairs_h[idx], sub_off, sub_seeds,
                             x_scalar=25, min_dist=17, max_seeds=1, k=17)
    for f in ("score", "status", "seed_idx", "n_kept"):
        assert np.array_equal(got[f][idx], ref[f]), f
    for f in ("beg", "end"):
        assert np.array_equal(got[f][idx].view(np.uint32), ref[f].astype(np.uint32)), f
    assert np.array_equal(got["cells"][idx].astype(np.uint64), ref["cells"].astype(np.uint64))


# ---- both strands ----------------------------------------------------------------

def _revcomp(s):
    return (3 - np.asarray(s, np.uint8)[::-1]).astype(np.uint8)


def gpu2(codes, off, length, k, m, bloom_bits=0):
    with xd.ReadStore(codes, off, length) as st:
        r = xd.find_overlaps(st, k=k, m=m, bloom_bits=bloom_bits, strands=2)
    torch.cuda.synchronize()
    return (r["pairs"].cpu().numpy().view(np.uint32).reshape(-1, 2),
            r["seed_off"].cpu().numpy().view(np.uint64),
            r["seeds"].cpu().numpy().view(np.uint32).reshape(-1, 2), r["counts"],
            r["rc"].cpu().numpy())


def assert_same2(got, ref, label):
    assert_same(got, ref, label)
    assert np.array_equal(got[4], ref[4]), "%s: rc differs" % label


def test_both_strands_small_sets_match_oracle():
    rng = np.random.default_rng(22)
    for trial in range(30):
        base = rng.integers(0, 4, 3000).astype(np.uint8)
        seqs = []
        for _ in range(int(rng.integers(1, 30))):
            n = int(rng.integers(0, 500))
            s = int(rng.integers(0, 3000 - n + 1))
            r = base[s:s + n].copy()
            flip = rng.random(n) < 0.04
            r[flip] = rng.integers(0, 4, int(flip.sum()))
            seqs.append(_revcomp(r) if rng.random() < 0.5 else r)
        if trial % 5 == 0:
            seqs.append(np.tile(np.array([0, 1, 2, 3], np.uint8), 30))  # ACGT...: palindromes
        k = int(rng.choice([1, 2, 4, 5, 11, 17, 31]))
        m = int(rng.choice([2, 3, 8, 64]))
        codes, off, length = _reads(seqs)
        ref = ov.find_overlaps(codes, off, length, k, 2, m, strands=2)
        got = gpu2(codes, off, length, k, m)
        assert_same2(got, ref, "trial %d (k=%d, m=%d, %d reads)" % (trial, k, m, len(seqs)))


def flipped_c2_small():
    """The c2-small read set with every other read stored reverse-complemented."""
    w = synth.config("c2-small")
    seqs = [w.read(r).copy() for r in range(w.n_reads)]
    seqs = [_revcomp(s) if r % 2 else s for r, s in enumerate(seqs)]
    return _reads(seqs)


def test_both_strands_on_opposite_strand_read_set():
    codes, off, length = flipped_c2_small()
    ref = ov.find_overlaps_sorted(codes, off, length, 17, 2, 8, strands=2)
    assert ref[4].sum() > 0.3 * ref[4].size      # opposite-strand pairs are common
    for bits in (0, 4):
        got = gpu2(codes, off, length, 17, 8, bloom_bits=bits)
        assert_same2(got, ref, "flipped c2-small bloom_bits=%d" % bits)
    # forward k-mers alone miss the opposite-strand overlaps
    fwd = gpu(codes, off, length, 17, 8)
    assert fwd[3]["pairs"] < ref[0].shape[0]
    # strands = 1 through the new entry point is the forward-only call
    with xd.ReadStore(codes, off, length) as st:
        r1 = xd.find_overlaps(st, k=17, m=8, strands=1)
        torch.cuda.synchronize()
        assert np.array_equal(r1["pairs"].cpu().numpy().view(np.uint32).reshape(-1, 2), fwd[0])
        assert np.array_equal(r1["seeds"].cpu().numpy().view(np.uint32).reshape(-1, 2), fwd[2])
        assert int(r1["rc"].sum()) == 0


def test_both_strands_pairs_feed_alignment():
    # candidate pairs from both strands, aligned with their strand flags, on
    # a sample of pairs against the pair oracle
    codes, off, length = flipped_c2_small()
    with xd.ReadStore(codes, off, length) as st:
        r = xd.find_overlaps(st, k=17, m=8, strands=2)
        P = r["counts"]["pairs"]
        out = xd.align_pairs(st, r["pairs"], r["seed_off"], r["seeds"], rc=r["rc"],
                             x_scalar=25, min_dist=17, max_seeds=1, k=17,
                             n_seeds=r["counts"]["seeds"])
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        so = r["seed_off"].cpu().numpy()
        pairs_h = r["pairs"].cpu().numpy()
        seeds_h = r["seeds"].cpu().numpy()
        rc_h = r["rc"].cpu().numpy()
    assert (got["status"] == 0).all()
    idx = np.linspace(0, P - 1, 60).astype(np.int64)
    idx = np.unique(np.concatenate([idx, np.flatnonzero(rc_h)[:30]]))
    sub_off = np.concatenate([[0], np.cumsum(so[idx + 1] - so[idx])]).astype(np.uint64)
    sub_seeds = np.concatenate([seeds_h[so[i]:so[i + 1]] for i in idx])
    ref = opairs.align_pairs(codes, off, length, pairs_h[idx], sub_off, sub_seeds,
                             rc=rc_h[idx], x_scalar=25, min_dist=17, max_seeds=1, k=17)
    for f in ("score", "status", "seed_idx", "n_kept"):
        assert np.array_equal(got[f][idx], ref[f]), f
    for f in ("beg", "end"):
        assert np.array_equal(got[f][idx].astype(np.uint32), ref[f].astype(np.uint32)), f
    assert np.array_equal(got["cells"][idx].astype(np.uint64), ref["cells"].astype(np.uint64))
    # true opposite-strand overlaps align over kilobases
    assert got["score"][rc_h == 1].max() > 1000
