"""Serving: requests admitted by HBM budget, packed into batches on several
streams; every request's results must be identical to aligning it alone."""
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402


def make_requests(w, rng, count, max_size):
    reqs = []
    for _ in range(count):
        n = int(np.exp(rng.uniform(0, np.log(max_size + 1))))
        n = max(1, min(n, w.n_tasks))
        s = int(rng.integers(0, w.n_tasks - n + 1))
        X = int(rng.choice([7, 25]))
        reqs.append((np.stack([w.ra[s:s + n], w.rb[s:s + n]], 1),
                     np.stack([w.pa[s:s + n], w.pb[s:s + n]], 1), X))
    return reqs


def alone(store, pairs, seeds, X, k):
    p = torch.from_numpy(pairs.astype(np.int32)).cuda()
    s = torch.from_numpy(seeds.astype(np.int32)).cuda()
    out = xd.align_batch(store, p, s, x=None, x_scalar=X, k=k)
    torch.cuda.synchronize()
    return {k2: v.cpu().numpy() for k2, v in out.items()}


def same(a, b):
    return (np.array_equal(a["score"], b["score"]) and np.array_equal(a["status"], b["status"])
            and np.array_equal(a["beg"].astype(np.uint32), b["beg"].astype(np.uint32))
            and np.array_equal(a["end"].astype(np.uint32), b["end"].astype(np.uint32))
            and np.array_equal(a["cells"].astype(np.uint64), b["cells"].astype(np.uint64)))


def test_server_mix_equals_alone():
    w = synth.config("c5-small")
    rng = np.random.default_rng(3)
    reqs = make_requests(w, rng, 80, 600)
    store = xd.ReadStore.from_workload(w)
    ref = [alone(store, p, s, X, w.k) for (p, s, X) in reqs]
    fixed = xd.server_fixed_bytes(store, slots=3)
    budget = fixed + 4 * xd.request_bytes(600)
    srv = xd.Server(store, hbm_budget_bytes=budget, slots=3, max_batch_tasks=900, k=w.k)
    ids = []
    for q, (p, s, X) in enumerate(reqs):
        ids.append(srv.submit(p, s, x_scalar=X))
        if q % 3 == 0:
            time.sleep(0.0005 * rng.random())
    got = [srv.poll(i, timeout_ms=-1) for i in ids]
    st = srv.stats()
    srv.close()
    for q, (g, r) in enumerate(zip(got, ref)):
        assert same(g, r), "request %d differs from its solo run" % q
        assert g["info"]["t_done"] >= g["info"]["t_start"] >= g["info"]["t_submit"]
    assert st["completed"] == len(reqs)
    assert st["peak_inflight_bytes"] <= budget - fixed
    assert st["batches"] < len(reqs)          # requests were packed together
    assert st["peak_busy_slots"] >= 2         # batches overlapped on the device
    # and the solo runs agree with the oracle on a sample
    for q in range(0, len(reqs), 9):
        p, s, X = reqs[q]
        o, _ = oracle.align_batch(w.codes, w.off, w.length, p, s, x_scalar=X, k=w.k)
        assert same(got[q], o)
    store.close()


def test_server_cancel_zero_and_oversize():
    w = synth.config("c5-small")
    store = xd.ReadStore.from_workload(w)
    fixed = xd.server_fixed_bytes(store, slots=1)
    assert fixed > 0
    with pytest.raises(xd.XdropError):  # nothing left for requests
        xd.Server(store, hbm_budget_bytes=fixed, slots=1, k=w.k)
    srv = xd.Server(store, hbm_budget_bytes=fixed + xd.request_bytes(300), slots=1, k=w.k)
    p = np.stack([w.ra[:300], w.rb[:300]], 1)
    s = np.stack([w.pa[:300], w.pb[:300]], 1)
    a = srv.submit(p, s, x_scalar=25)
    b = srv.submit(p, s, x_scalar=25)        # waits: the budget holds one
    srv.cancel(b)
    z = srv.submit(p[:0], s[:0], x_scalar=25)
    assert srv.poll(z, timeout_ms=-1)["score"].size == 0
    with pytest.raises(xd.XdropError):
        srv.submit(np.zeros((301, 2), np.uint32), np.zeros((301, 2), np.uint32), x_scalar=5)
    ra = srv.poll(a, timeout_ms=-1)
    assert same(ra, alone(store, p, s, 25, w.k))
    st = srv.stats()
    assert st["cancelled"] == 1
    srv.close()
    store.close()
