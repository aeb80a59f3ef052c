"""GPU parity for banded Smith-Waterman (xd_banded_batch) against the oracle
(oracle/banded_oracle.c), element by element: score, end cell, status,
cells."""
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


def run(w, ws, scheme=(1, -1, -1)):
    store = xd.ReadStore.from_workload(w)
    try:
        pairs, seeds, _ = xd.workload_tensors(w, "cuda")
        wt = torch.from_numpy(np.ascontiguousarray(ws, np.int32)).cuda()
        out = xd.banded_batch(store, pairs, seeds, w=wt, k=w.k, match=scheme[0],
                              mismatch=scheme[1], gap=scheme[2])
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        store.close()
    ref = oracle.banded_batch(w.codes, w.off, w.length, np.stack([w.ra, w.rb], 1),
                              np.stack([w.pa, w.pb], 1), ws, k=w.k, match=scheme[0],
                              mismatch=scheme[1], gap=scheme[2])
    return got, ref


def assert_same(got, ref, label):
    for key in ("status", "score"):
        bad = np.nonzero(got[key] != ref[key])[0]
        assert bad.size == 0, "%s %s at %s: gpu %s oracle %s" % (label, key, bad[:5],
                                                               got[key][bad[:5]], ref[key][bad[:5]])
    bad = np.nonzero((got["end"].view(np.uint32) != ref["end"]).any(1))[0]
    assert bad.size == 0, "%s end at %s: gpu %s oracle %s" % (label, bad[:5],
                                                           got["end"][bad[:5]], ref["end"][bad[:5]])
    assert np.array_equal(got["cells"].view(np.uint64), ref["cells"]), label


@pytest.mark.parametrize("wdt", [0, 1, 8, 31, 48])
def test_banded_c2_small(wdt):
    w = synth.config("c2-small")
    got, ref = run(w, np.full(w.n_tasks, wdt, np.int32))
    assert (ref["status"] == 0).all()
    assert_same(got, ref, "w=%d" % wdt)


def edge_banded():
    rng = np.random.default_rng(8)
    A = rand_codes(rng, 3000)
    B = mutate_codes(rng, A, 0.15)
    C = rand_codes(rng, 2000)
    S = rand_codes(rng, 40)
    reads = [A, B, C, S, A[:17].copy()]
    tasks = [(0, 1, 1500, 1480, 0), (0, 1, 0, 0, 0), (0, 1, 2983, 2900, 0),
             (0, 2, 100, 1900, 0), (2, 0, 1900, 100, 0),   # far off the main diagonal
             (0, 3, 5, 20, 0), (3, 0, 20, 5, 0), (4, 0, 0, 0, 0), (0, 4, 2983, 0, 0),
             (0, 1, 10, 10, 0), (0, 9, 1, 1, 0), (0, 1, 2990, 5, 0)]
    return workload_from(reads, tasks)


def test_banded_edges_and_statuses():
    w = edge_banded()
    ws = np.array([24, 48, 48, 48, 48, 10, 10, 5, 48, 49, 8, 8], np.int32)
    got, ref = run(w, ws)
    assert ref["status"][9] == oracle.TASK_BAD_X and ref["status"][10] == oracle.TASK_BAD_READ
    assert ref["status"][11] == oracle.TASK_BAD_SEED
    assert_same(got, ref, "edges")


@pytest.mark.parametrize("scheme", [(2, -3, -2), (1, -1, -3), (5, -4, -7)])
def test_banded_scoring(scheme):
    w = synth.config("c1-small")
    got, ref = run(w, np.full(w.n_tasks, 20, np.int32), scheme)
    assert_same(got, ref, "scheme %s" % (scheme,))


def test_banded_scalar_band_width():
    # the scalar w_scalar form (no per-task array), with an odd task count
    w = synth.config("c2-small")
    w = w.subset(np.arange(w.n_tasks - (1 - w.n_tasks % 2)))
    store = xd.ReadStore.from_workload(w)
    try:
        pairs, seeds, _ = xd.workload_tensors(w, "cuda")
        for wdt in (0, 16, 21):
            out = xd.banded_batch(store, pairs, seeds, w=None, w_scalar=wdt, k=w.k)
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in out.items()}
            ref = oracle.banded_batch(w.codes, w.off, w.length, np.stack([w.ra, w.rb], 1),
                                      np.stack([w.pa, w.pb], 1),
                                      np.full(w.n_tasks, wdt, np.int32), k=w.k)
            assert_same(got, ref, "scalar w=%d" % wdt)
    finally:
        store.close()
