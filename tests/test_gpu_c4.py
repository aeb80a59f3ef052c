"""Full-size run of the largest workload, one GPU's share of a 100 Mbp genome
(c4: 20,000,000 (pair, seed) tasks over a 30x read set with repeat copies,
10 % of the tasks spurious, X = 25), in the batched form: every task checked
against properties that hold at any size and against the plain form, a
sample (true and spurious tasks) element by element against the oracle.
Generating the read set takes about two minutes on one host core."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402


def test_c4_batched_full_size():
    print("generating c4", flush=True)
    w = synth.config("c4")
    print("c4: %d reads, %d tasks" % (len(w.length), w.n_tasks), flush=True)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    out = xd.align_batch(store, pairs, seeds, x=x, k=w.k, persistent=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    print("c4 batched form done", flush=True)
    out = xd.align_batch(store, pairs, seeds, x=x, k=w.k)
    torch.cuda.synchronize()
    plain = {k: v.cpu().numpy() for k, v in out.items()}
    store.close()
    del out, pairs, seeds, x
    for key in got:
        assert np.array_equal(got[key], plain[key]), "plain and batched forms differ: " + key
    # every task: valid, seed inside the alignment, score at least the seed
    assert (got["status"] == 0).all()
    assert (got["score"] >= w.k).all()
    beg, end = got["beg"].astype(np.int64), got["end"].astype(np.int64)
    assert (beg[:, 0] <= w.pa).all() and (end[:, 0] >= w.pa.astype(np.int64) + w.k).all()
    assert (beg[:, 1] <= w.pb).all() and (end[:, 1] >= w.pb.astype(np.int64) + w.k).all()
    assert (end[:, 0] <= w.length[w.ra]).all() and (end[:, 1] <= w.length[w.rb]).all()
    # 10 % of the tasks are spurious (reads over different copies of one
    # repeat segment).  Their alignments need not stop at the segment's end:
    # with +1/-1/-1 the best alignment of unrelated DNA loses score only very
    # slowly, so X = 25 can carry them far into the flanks.
    spur = w.spurious.astype(bool)
    assert spur.sum() == w.n_tasks // 10
    # sampled tasks, element by element: 1,200 true and 300 spurious
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(np.nonzero(~spur)[0], 1200, replace=False),
                          rng.choice(np.nonzero(spur)[0], 300, replace=False)])
    ref = oracle.align_workload(w.subset(idx))
    for key in ("score", "status"):
        assert np.array_equal(got[key][idx], ref[key]), key
    assert np.array_equal(got["beg"][idx].astype(np.uint32), ref["beg"])
    assert np.array_equal(got["end"][idx].astype(np.uint32), ref["end"])
    assert np.array_equal(got["cells"][idx].astype(np.uint64), ref["cells"])
