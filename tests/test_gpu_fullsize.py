"""Full-size parity on the workload the benchmark times (c2: 100,000 read
pairs from a 30x 4.6 Mbp read set, X = 25), in the same launch form: sampled
tasks are checked one by one against the oracle, every task against
properties that hold at any size."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402


@pytest.fixture(scope="module")
def c2():
    print("generating c2", flush=True)
    return synth.config("c2")


def test_c2_sampled_parity_and_invariants(c2):
    w = c2
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    out = xd.align_batch(store, pairs, seeds, x=x, k=w.k)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    store.close()
    # every task: valid, seed inside the alignment, score at least the seed
    assert (got["status"] == 0).all()
    assert (got["score"] >= w.k).all()
    beg, end = got["beg"].astype(np.int64), got["end"].astype(np.int64)
    assert (beg[:, 0] <= w.pa).all() and (end[:, 0] >= w.pa.astype(np.int64) + w.k).all()
    assert (beg[:, 1] <= w.pb).all() and (end[:, 1] >= w.pb.astype(np.int64) + w.k).all()
    assert (end[:, 0] <= w.length[w.ra]).all() and (end[:, 1] <= w.length[w.rb]).all()
    assert (got["cells"] > 0).all()
    # sampled tasks, element by element
    idx = np.random.default_rng(0).choice(w.n_tasks, 1500, replace=False)
    sub = w.subset(idx)
    ref = oracle.align_workload(sub)
    for key in ("score", "status"):
        assert np.array_equal(got[key][idx], ref[key]), key
    assert np.array_equal(got["beg"][idx].astype(np.uint32), ref["beg"])
    assert np.array_equal(got["end"][idx].astype(np.uint32), ref["end"])
    assert np.array_equal(got["cells"][idx].astype(np.uint64), ref["cells"])
