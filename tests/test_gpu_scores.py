"""GPU parity across the whole scoring range the X-drop calls accept
(|match|, |mismatch|, |gap| up to 1000): the HIP path against the CPU oracle,
element by element.

Match bonuses above a byte take the general kernels (match indicator times
the bonus); long extensions with large scores pass the U rebase, which the
window tiers and the band tier each do on their own.
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
from paper_2001_10049_amd import _lib  # noqa: E402
from test_gpu_parity import assert_same, band_workload, edge_workload  # noqa: E402

SCHEMES = [(200, -300, -150), (1000, -1000, -1000), (127, -127, -127), (127, 126, -1),
           (10, 5, -1), (1, -1000, -1), (1, -1, -1000), (1000, 999, -1), (2, -1000, -3)]


def scaled_x(w, f):
    """X of every valid task times f (capped at X_MAX); invalid X kept."""
    x = w.x.astype(np.int64)
    ok = (x >= 0) & (x <= _lib.X_MAX)
    x[ok] = np.minimum(x[ok] * f, _lib.X_MAX)
    return x.astype(np.int32)


def run(w, x, scheme, form):
    M, MM, G = scheme
    store = xd.ReadStore.from_workload(w)
    try:
        pairs, seeds, _ = xd.workload_tensors(w, "cuda")
        xs = torch.from_numpy(x).to("cuda")
        out = xd.align_batch(store, pairs, seeds, x=xs, k=w.k, match=M, mismatch=MM, gap=G,
                             persistent=form == "persistent")
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        store.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
@pytest.mark.parametrize("scheme", SCHEMES, ids=lambda s: "%d_%d_%d" % s)
def test_edge_workload_wide_scores(scheme, form):
    print("edge", scheme, form, flush=True)
    w = edge_workload()
    x = scaled_x(w, scheme[0])
    M, MM, G = scheme
    ref = oracle.align_workload(w, x=x, match=M, mismatch=MM, gap=G)
    assert_same(run(w, x, scheme, form), ref, label="edge %s %s" % (scheme, form))


@pytest.mark.parametrize("scheme", [(200, -300, -150), (1000, -1000, -1000), (1, -1000, -1),
                                    (127, 126, -1)], ids=lambda s: "%d_%d_%d" % s)
def test_c2_small_wide_scores(scheme):
    w = synth.config("c2-small")
    w = w.subset(np.arange(min(400, w.n_tasks)))
    x = scaled_x(w, scheme[0])
    M, MM, G = scheme
    ref = oracle.align_workload(w, x=x, match=M, mismatch=MM, gap=G)
    assert (ref["status"] == 0).all()
    for form in ("plain", "persistent"):
        print("c2-small", scheme, form, flush=True)
        assert_same(run(w, x, scheme, form), ref, label="c2-small %s %s" % (scheme, form))


@pytest.mark.parametrize("scheme", [(200, -300, -150), (1000, -1000, -1000)],
                         ids=lambda s: "%d_%d_%d" % s)
def test_band_tier_wide_scores(scheme):
    w = band_workload()
    x = scaled_x(w, scheme[0])
    M, MM, G = scheme
    print("band", scheme, flush=True)
    ref = oracle.align_workload(w, x=x, match=M, mismatch=MM, gap=G)
    assert_same(run(w, x, scheme, "plain"), ref, label="band %s" % (scheme,))


def long_pair_workload(length, p_err, seed):
    """A read, an identical copy and a mutated copy of it, with seeds at the
    start: extensions over the whole read."""
    rng = np.random.default_rng(seed)
    A = rand_codes(rng, length)
    B = mutate_codes(rng, A, p_err)
    reads = [A, A.copy(), B]
    # a shared 17-mer near the start of A and B
    idx = {bytes(A[i:i + 17]): i for i in range(0, 2000)}
    j0 = next(j for j in range(0, 2000) if bytes(B[j:j + 17]) in idx)
    return reads, idx[bytes(B[j0:j0 + 17])], j0


@pytest.mark.parametrize("scheme,length,X", [((1000, -1000, -1000), 400_000, 30_000),
                                              ((1, -1, -1000), 600_000, 3)],
                         ids=["large_scores", "unit_large_gap"])
def test_window_rebase(scheme, length, X):
    # U grows by about match/2 + g per antidiagonal: these extensions pass
    # 2^30 and are rebased on the way; identical reads give the closed form
    # score = match * length
    reads, pa, pb = long_pair_workload(length, 0.01, 5)
    M, MM, G = scheme
    tasks = [(0, 1, 0, 0, X), (0, 1, length // 2, length // 2, X), (0, 2, pa, pb, 20 * X)]
    w = workload_from(reads, tasks)
    ref = oracle.align_workload(w, match=M, mismatch=MM, gap=G)
    assert ref["score"][0] == M * length and ref["score"][1] == M * length
    for form in ("plain", "persistent"):
        print("rebase", scheme, form, flush=True)
        assert_same(run(w, w.x, scheme, form), ref, label="rebase %s %s" % (scheme, form))


def test_band_tier_rebase():
    # identical 700 kbp reads, (1000, -1000, -300), X = 2^20: a cell k rows
    # off the diagonal scores 800 k below it, so the live band is about 1311
    # rows wide (band tier), and U (rising 800 per antidiagonal) passes 2^30
    # after about 1.34 M of the 1.4 M antidiagonals
    length = 700_000
    rng = np.random.default_rng(6)
    A = rand_codes(rng, length)
    w = workload_from([A, A.copy()], [(0, 1, 0, 0, 1 << 20)])
    scheme = (1000, -1000, -300)
    ref = oracle.align_workload(w, match=1000, mismatch=-1000, gap=-300)
    assert ref["score"][0] == 1000 * length
    xd.profile_enable(True)
    xd.profile_read(reset=True)
    got = run(w, w.x, scheme, "plain")
    prof = xd.profile_read(reset=True)
    xd.profile_enable(False)
    assert prof["to_band"] == 1, prof
    assert_same(got, ref, label="band rebase")


def test_score_range_against_the_longest_read():
    # every score must fit an int32: match * longest read <= 2^31 - 1
    rng = np.random.default_rng(8)
    L = 2_200_000
    w = workload_from([rand_codes(rng, L), rand_codes(rng, 100)], [])
    store = xd.ReadStore.from_workload(w)
    lib = _lib.load()
    try:
        limit = (2 ** 31 - 1) // L
        for match, ok in ((limit, True), (limit + 1, False)):
            rc = lib.xd_align_batch(store.handle, None, None, None, 25, 0, 17, match, -1, -1,
                                    None, None, None, None, None, None)
            assert (rc == _lib.XD_OK) == ok, (match, rc)
            if not ok:
                assert b"2^31" in lib.xd_last_error()
    finally:
        store.close()
