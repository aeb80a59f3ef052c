"""Every task of the full-size workloads c2, c3, c4 and c5 against the oracle.

The oracle's results for each workload were recorded once as chunked SHA-256
digests by tests/golden/make_oracle_digests.py (a script that runs only the
oracle and the seeded generator); the GPU's results must reproduce every
chunk's digest, i.e. every score, coordinate, status and cell count.  A
differing chunk is rerun through the oracle to name the tasks."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from digest import CHUNK, input_digest, result_digests  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402

DIGESTS = json.load(open(os.path.join(HERE, "golden", "oracle_digests.json")))


def check_against_record(w, got, rec, label):
    assert input_digest(w) == rec["input"], "%s: generated inputs differ from the record" % label
    mine = result_digests(got, rec["chunk"])
    bad = [i for i, (a, b) in enumerate(zip(mine, rec["chunks"])) if a != b]
    if bad:
        lo = bad[0] * CHUNK
        idx = np.arange(lo, min(lo + CHUNK, w.n_tasks))
        ref = oracle.align_workload(w.subset(idx))
        diff = np.nonzero((got["score"][idx] != ref["score"]) |
                          (got["cells"][idx].astype(np.uint64) != ref["cells"]))[0]
        raise AssertionError("%s: %d of %d chunks differ; first chunk %d, tasks %s" % (
            label, len(bad), len(mine), bad[0], (idx[diff[:5]]).tolist()))
    assert int(got["cells"].astype(np.uint64).sum()) == rec["cells"]
    assert int(got["score"].astype(np.int64).sum()) == rec["score_sum"]


@pytest.mark.parametrize("name,forms", [("c2", ("plain", "persistent")), ("c3", ("persistent",)),
                                        ("c5", ("persistent",)), ("c4", ("persistent",))])
def test_every_task_matches_oracle_record(name, forms):
    if name not in DIGESTS:
        pytest.skip("no oracle record for %s" % name)
    print("generating", name, flush=True)
    w = synth.config(name)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, x = xd.workload_tensors(w, "cuda")
    try:
        for form in forms:
            print(name, form, w.n_tasks, "tasks", flush=True)
            out = xd.align_batch(store, pairs, seeds, x=x, k=w.k, persistent=form == "persistent")
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in out.items()}
            check_against_record(w, got, DIGESTS[name], "%s %s" % (name, form))
    finally:
        store.close()
