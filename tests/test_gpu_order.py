"""Order independence: permuting the tasks permutes the results and changes
nothing else, in the plain and the batched forms (the longest-first queue,
the overflow lists and the persistent waves see a different order)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402


@pytest.mark.parametrize("name", ["c3-small", "c4-small"])
def test_permuted_tasks_give_permuted_results(name):
    w = synth.config(name)
    perm = np.random.default_rng(11).permutation(w.n_tasks)
    store = xd.ReadStore.from_workload(w)
    try:
        pairs, seeds, x = xd.workload_tensors(w, "cuda")
        p = torch.from_numpy(perm).cuda()
        for persistent in (False, True):
            a = xd.align_batch(store, pairs, seeds, x=x, k=w.k, persistent=persistent)
            b = xd.align_batch(store, pairs[p].contiguous(), seeds[p].contiguous(),
                               x=x[p].contiguous(), k=w.k, persistent=persistent)
            torch.cuda.synchronize()
            for key in a:
                assert torch.equal(a[key][p], b[key]), (name, persistent, key)
    finally:
        store.close()
