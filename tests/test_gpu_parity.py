"""GPU parity: the HIP path against the CPU oracle, element by element.

Every integer output (score, begin/end coordinates, status, evaluated cells)
must be identical.  Inputs are seeded synthetic workloads (synth) and
explicit edge cases.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import mutate_codes, rand_codes, workload_from

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402


def run_gpu(w, match=1, mismatch=-1, gap=-1, x=None, x_scalar=0, stream=None):
    store = xd.ReadStore.from_workload(w)
    try:
        pairs, seeds, xs = xd.workload_tensors(w, "cuda")
        out = xd.align_batch(store, pairs, seeds, x=xs if x is None else x, x_scalar=x_scalar,
                             k=w.k, match=match, mismatch=mismatch, gap=gap, stream=stream)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        store.close()


def assert_same(got, ref, idx=None, label=""):
    sel = slice(None) if idx is None else idx
    for key in ("status", "score"):
        g, r = got[key][sel], ref[key] if idx is None else ref[key]
        bad = np.nonzero(g != r)[0]
        assert bad.size == 0, "%s %s differs at %s: gpu %s oracle %s" % (
            label, key, bad[:5], g[bad[:5]], r[bad[:5]])
    for key in ("beg", "end"):
        g = got[key][sel].astype(np.uint32)
        r = ref[key]
        bad = np.nonzero((g != r).any(1))[0]
        assert bad.size == 0, "%s %s differs at %s: gpu %s oracle %s" % (
            label, key, bad[:5], g[bad[:5]], r[bad[:5]])
    g = got["cells"][sel].astype(np.uint64)
    bad = np.nonzero(g != ref["cells"])[0]
    assert bad.size == 0, "%s cells differ at %s: gpu %s oracle %s" % (
        label, bad[:5], g[bad[:5]], ref["cells"][bad[:5]])


@pytest.mark.parametrize("name", ["c1", "c1-small", "c2-small", "c3-small", "c4-small"])
def test_workload_parity(name):
    print("parity", name, flush=True)
    w = synth.config(name)
    got = run_gpu(w)
    ref = oracle.align_workload(w)
    assert (ref["status"] == 0).all()
    assert_same(got, ref, label=name)


@pytest.mark.parametrize("scoring", [(2, -3, -2), (1, -2, -1), (3, -1, -2), (5, -4, -1)])
def test_scoring_variants(scoring):
    M, MM, G = scoring
    print("scoring", scoring, flush=True)
    w = synth.config("c2-small")
    w = w.subset(np.arange(0, w.n_tasks, 3))
    got = run_gpu(w, M, MM, G)
    ref = oracle.align_workload(w, match=M, mismatch=MM, gap=G)
    assert_same(got, ref, label=str(scoring))


@pytest.mark.parametrize("X", [0, 1, 3, 100])
def test_x_values(X):
    print("X", X, flush=True)
    w = synth.config("c2-small")
    w = w.subset(np.arange(0, w.n_tasks, 5))
    xs = np.full(w.n_tasks, X, np.int32)
    w.x = xs
    got = run_gpu(w)
    ref = oracle.align_workload(w)
    assert_same(got, ref, label="X=%d" % X)


def test_scalar_x():
    w = synth.config("c1-small")
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, _ = xd.workload_tensors(w, "cuda")
    out = xd.align_batch(store, pairs, seeds, x=None, x_scalar=11, k=w.k)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    store.close()
    ref = oracle.align_workload(w, x=np.full(w.n_tasks, 11, np.int32))
    assert_same(got, ref, label="x_scalar")


def edge_workload():
    rng = np.random.default_rng(7)
    reads, tasks = [], []
    A = rand_codes(rng, 3000)
    reads += [A, A.copy()]                      # 0, 1 identical
    B = mutate_codes(rng, A, 0.15)
    reads += [B]                                # 2 noisy copy of A
    K = rand_codes(rng, 17)
    reads += [K, K.copy()]                      # 3, 4 reads of length k
    U = rand_codes(rng, 2500)
    reads += [U]                                # 5 unrelated
    C = A[1000:2200].copy()
    reads += [C]                                # 6 contained in A
    E = np.concatenate([rand_codes(rng, 500), A[:17]])
    reads += [E]                                # 7 seed at its end
    # identical, several X (narrow to wide bands)
    for X in (0, 1, 7, 25, 50, 200, 600, 1200):
        tasks.append((0, 1, 1000, 1000, X))
    # seed at the start / end of both reads
    tasks += [(0, 1, 0, 0, 25), (0, 1, 3000 - 17, 3000 - 17, 25)]
    tasks += [(3, 4, 0, 0, 25), (3, 4, 0, 0, 0)]
    tasks += [(0, 7, 0, 500, 25), (7, 0, 500, 0, 25)]
    tasks += [(0, 6, 1500, 500, 25), (6, 0, 500, 1500, 40)]
    # noisy copy: find a shared 17-mer by brute force
    sa = {bytes(A[i:i + 17]): i for i in range(0, 3000 - 17)}
    for j in range(0, len(B) - 17):
        i = sa.get(bytes(B[j:j + 17]))
        if i is not None and 800 < i < 2200:
            tasks += [(0, 2, i, j, 7), (0, 2, i, j, 25), (2, 0, j, i, 50), (0, 2, i, j, 300)]
            break
    # unrelated reads with a planted shared k-mer: early X-drop exit
    tasks += [(0, 5, 100, 100, 25)]
    reads[5][100:117] = A[100:117]
    # non-exact seed (scored ungapped)
    tasks += [(0, 5, 2000, 2000, 10)]
    # invalid tasks
    tasks += [(0, 99, 0, 0, 25), (99, 0, 0, 0, 25), (0, 1, 2990, 0, 25), (0, 1, 0, 2984, 25),
              (0, 1, 5, 5, -1), (0, 1, 5, 5, (1 << 20) + 1)]
    return workload_from(reads, tasks)


def test_edge_cases():
    w = edge_workload()
    got = run_gpu(w)
    ref = oracle.align_workload(w)
    assert_same(got, ref, label="edge")


def band_workload():
    """Extensions whose live band outgrows the 1024-cell window, beside narrow ones."""
    rng = np.random.default_rng(9)
    A = rand_codes(rng, 3000)
    L = rand_codes(rng, 20000)
    R1, R2 = rand_codes(rng, 5000), rand_codes(rng, 5000)
    M = mutate_codes(rng, A, 0.15)
    reads = [A, A.copy(), L, L.copy(), R1, R2, M]
    tasks = [(0, 1, 1500, 1500, 4000),         # identical, band grows to the read ends
             (0, 1, 1500, 1500, 25),           # same pair, narrow
             (2, 3, 10000, 10000, 2000),       # identical 20 kbp, ~2700-cell band
             (4, 5, 2500, 2500, 1 << 20),      # unrelated reads, no pruning: full grid
             (0, 6, 1000, 1000, 1500),         # 15 % mutated copy, wide X
             (2, 3, 0, 19000, 1 << 20),        # seed at both read ends
             (0, 1, 0, 0, 3000)]
    return workload_from(reads, tasks)


@pytest.mark.parametrize("form", ["plain", "persistent", "persistent1", "plan"])
def test_band_tier_parity(form):
    # bands wider than 1024 cells run in the band tier: same results as the oracle
    w = band_workload()
    print("band tier", form, flush=True)
    ref = oracle.align_workload(w)
    xd.profile_enable(True)
    xd.profile_read(reset=True)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, xs = xd.workload_tensors(w, "cuda")
    if form == "plan":
        plan = xd.Plan(store, pairs, seeds, x=xs, k=w.k)
        out = plan.launch()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        plan.close()
    else:
        tuning = dict(band_blocks=1) if form == "persistent1" else None
        out = xd.align_batch(store, pairs, seeds, x=xs, k=w.k, persistent=form != "plain",
                             tuning=tuning)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    prof = xd.profile_read(reset=True)
    xd.profile_enable(False)
    store.close()
    assert (ref["status"] == 0).all()
    assert_same(got, ref, label="band " + form)
    if form != "plan":  # plans record no profile
        assert prof["to_band"] >= 6, prof


def test_band_tier_scoring():
    w = band_workload().subset(np.array([0, 4, 6]))
    for (M, MM, G) in ((2, -3, -2), (5, -4, -7)):
        got = run_gpu(w, match=M, mismatch=MM, gap=G)
        assert_same(got, oracle.align_workload(w, match=M, mismatch=MM, gap=G),
                    label="band %s" % ((M, MM, G),))


def test_empty_batch():
    w = synth.config("c1-small")
    store = xd.ReadStore.from_workload(w)
    e = torch.empty((0, 2), dtype=torch.int32, device="cuda")
    out = xd.align_batch(store, e, e, x=None, x_scalar=5, k=17)
    torch.cuda.synchronize()
    assert out["score"].numel() == 0
    store.close()


def test_repeatable_and_order_independent():
    w = synth.config("c2-small")
    a = run_gpu(w)
    perm = np.random.default_rng(3).permutation(w.n_tasks)
    b = run_gpu(w.subset(perm))
    for key in ("score", "status", "beg", "end", "cells"):
        assert np.array_equal(a[key][perm], b[key]), key


def test_store_info():
    w = synth.config("c1-small")
    with xd.ReadStore.from_workload(w) as s:
        info = s.info()
    assert info["n_reads"] == w.n_reads and info["max_len"] == int(w.length.max())


TUNINGS = [dict(), dict(waves_per_cu=8, group_steps=4), dict(waves_per_cu=16, group_steps=16),
           dict(order=2, group_steps=8), dict(x_tier1=5, x_tier2=30),
           dict(x_tier1=1000, x_tier2=1000)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: str(sorted(t.items())))
@pytest.mark.parametrize("name", ["c2-small", "c3-small", "c4-small"])
def test_persistent_parity(name, tuning):
    print("persistent", name, tuning, flush=True)
    w = synth.config(name)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    out = xd.align_batch(store, pairs, seeds, x=x, k=w.k, persistent=True, tuning=tuning)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    store.close()
    assert_same(got, oracle.align_workload(w), label="persistent " + name)


@pytest.mark.parametrize("wl", ["edge", "band", "flank"])
def test_packed_128_window_parity(wl):
    # every extension with 1 < X <= 5000 starts in the 128-cell window, which
    # the batched form runs in the packed two-extension kernel for +1/-1/-1:
    # walls, reads of length k, early exits, X up to its limit and past it,
    # bands that outgrow it (their state resumes in the 256-cell window)
    w = {"edge": edge_workload, "band": band_workload, "flank": random_flank_workload}[wl]()
    print("packed 128", wl, flush=True)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    out = xd.align_batch(store, pairs, seeds, x=x, k=w.k, persistent=True,
                         tuning=dict(x_tier1=1, x_tier2=5000))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    store.close()
    assert_same(got, oracle.align_workload(w), label="packed 128 " + wl)


@pytest.mark.parametrize("wl", ["edge", "band", "flank"])
def test_packed_256_window_parity(wl):
    # every extension with X > 1 starts in the 256-cell window: the packed
    # four-rows-per-lane kernel from a seed (not from a saved state) for
    # X <= 4096, the 32-bit kernel past that; bands that outgrow 256 rows
    # leave their state for the 512-cell window
    w = {"edge": edge_workload, "band": band_workload, "flank": random_flank_workload}[wl]()
    print("packed 256", wl, flush=True)
    xd.profile_enable(True)
    xd.profile_read(reset=True)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    out = xd.align_batch(store, pairs, seeds, x=x, k=w.k, persistent=True,
                         tuning=dict(x_tier1=1, x_tier2=1))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    prof = xd.profile_read(reset=True)
    xd.profile_enable(False)
    store.close()
    assert_same(got, oracle.align_workload(w), label="packed 256 " + wl)
    # nothing started below the 256-cell window
    assert prof["to_tier2"] == 0 and prof["to_tier3"] == 0, prof


def test_persistent_edge_and_scoring():
    w = edge_workload()
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    for (M, MM, G) in ((1, -1, -1), (2, -3, -2)):
        out = xd.align_batch(store, pairs, seeds, x=x, k=w.k, match=M, mismatch=MM, gap=G,
                             persistent=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        assert_same(got, oracle.align_workload(w, match=M, mismatch=MM, gap=G),
                    label="edge persistent %s" % ((M, MM, G),))
    store.close()


def test_plan_replays_and_input_rewrites():
    w = synth.config("c3-small")
    ref = oracle.align_workload(w)
    perm = np.random.default_rng(5).permutation(w.n_tasks)
    ref_perm = {k: v[perm] for k, v in ref.items()}
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    pairs_p, seeds_p, x_p = xd.workload_tensors(w.subset(perm), "cuda")
    plan = xd.Plan(store, pairs, seeds, x=x, k=w.k)
    orig = (pairs.clone(), seeds.clone(), x.clone())
    for rep in range(4):
        # eager work and a synchronisation between replays
        junk = torch.arange(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        if rep % 2:
            pairs.copy_(pairs_p), seeds.copy_(seeds_p), x.copy_(x_p)
            expect = ref_perm
        else:
            pairs.copy_(orig[0]), seeds.copy_(orig[1]), x.copy_(orig[2])
            expect = ref
        out = plan.launch()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        assert_same(got, expect, label="replay %d" % rep)
        del junk
    plan.close()
    store.close()


def random_flank_workload(n_pairs=300, length=6000, seed=21):
    """Unrelated read pairs sharing one planted 17-mer: every extension runs
    into random sequence, where X = 25 bands widen to 100-400 cells."""
    rng = np.random.default_rng(seed)
    reads, tasks = [], []
    for p in range(n_pairs):
        a, b = rand_codes(rng, length), rand_codes(rng, length)
        pa, pb = int(rng.integers(0, length - 17)), int(rng.integers(0, length - 17))
        b[pb:pb + 17] = a[pa:pa + 17]
        reads += [a, b]
        tasks.append((2 * p, 2 * p + 1, pa, pb, (25, 50)[p % 2]))
    return workload_from(reads, tasks)


@pytest.mark.parametrize("form", ["plain", "persistent", "plan"])
def test_wide_windows_parity(form):
    # the 128-, 256- and 512-cell windows, reached by overflow
    w = random_flank_workload()
    print("wide windows", form, flush=True)
    ref = oracle.align_workload(w)
    xd.profile_enable(True)
    xd.profile_read(reset=True)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, xs = xd.workload_tensors(w, "cuda")
    if form == "plan":
        plan = xd.Plan(store, pairs, seeds, x=xs, k=w.k)
        out = plan.launch()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        plan.close()
    else:
        out = xd.align_batch(store, pairs, seeds, x=xs, k=w.k, persistent=form == "persistent")
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    prof = xd.profile_read(reset=True)
    xd.profile_enable(False)
    store.close()
    assert_same(got, ref, label="wide " + form)
    if form != "plan":
        assert prof["to_tier3"] > 0 and prof["to_tier4"] > 0, prof
        # most moves to a wider window resume from the narrower window's
        # state; past each window's share of state slots they re-run from
        # the seed (both paths are taken here)
        moves = sum(prof[f] for f in ("to_tier2", "to_tier3", "to_tier4", "to_tier5"))
        assert 0 < prof["resumed"] < moves, prof


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_wide_windows_general_scores(form):
    # the same flanks under +2/-3/-2 with X doubled (bands of the same widths:
    # 100-500 cells): the 32-bit kernels of every window, their saved states
    # and resumes, against the oracle
    w = random_flank_workload()
    w.x = (w.x * 2).astype(np.int32)
    print("wide windows +2/-3/-2", form, flush=True)
    ref = oracle.align_workload(w, match=2, mismatch=-3, gap=-2)
    xd.profile_enable(True)
    xd.profile_read(reset=True)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, xs = xd.workload_tensors(w, "cuda")
    out = xd.align_batch(store, pairs, seeds, x=xs, k=w.k, match=2, mismatch=-3, gap=-2,
                         persistent=form == "persistent")
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    prof = xd.profile_read(reset=True)
    xd.profile_enable(False)
    store.close()
    assert_same(got, ref, label="wide +2/-3/-2 " + form)
    assert prof["to_tier3"] > 0 and prof["to_tier4"] > 0, prof
    moves = sum(prof[f] for f in ("to_tier2", "to_tier3", "to_tier4", "to_tier5"))
    assert 0 < prof["resumed"] < moves, prof
