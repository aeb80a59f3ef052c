"""Batched form on the c3 workload (2,000,000 (pair, seed) tasks over the
30x 4.6 Mbp read set, X in {7, 25, 50}): identical results to the plain form
on every task, and sampled tasks identical to the oracle."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402


def test_c3_plain_vs_persistent_vs_plan():
    print("generating c3", flush=True)
    w = synth.config("c3")
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    a = xd.align_batch(store, pairs, seeds, x=x, k=w.k)
    b = xd.align_batch(store, pairs, seeds, x=x, k=w.k, persistent=True)
    plan = xd.Plan(store, pairs, seeds, x=x, k=w.k)
    c = plan.launch()
    torch.cuda.synchronize()
    A = {k: v.cpu().numpy() for k, v in a.items()}
    B = {k: v.cpu().numpy() for k, v in b.items()}
    C = {k: v.cpu().numpy() for k, v in c.items()}
    plan.close()
    store.close()
    for key in A:
        assert np.array_equal(A[key], B[key]), key
        assert np.array_equal(A[key], C[key]), key
    assert (A["status"] == 0).all()
    idx = np.random.default_rng(1).choice(w.n_tasks, 1500, replace=False)
    ref = oracle.align_workload(w.subset(idx))
    assert np.array_equal(A["score"][idx], ref["score"])
    assert np.array_equal(A["beg"][idx].astype(np.uint32), ref["beg"])
    assert np.array_equal(A["end"][idx].astype(np.uint32), ref["end"])
    assert np.array_equal(A["cells"][idx].astype(np.uint64), ref["cells"])
