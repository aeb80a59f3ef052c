"""GPU parity for banded Smith-Waterman with traceback (xd_banded_traceback)
against the oracle (xo_banded_trace in oracle/banded_oracle.c): score, begin
and end cells, cells, status and the run-length path, element by element;
sub-batching by trace budget; the op-capacity status; and the full c2 batch
against the untraced kernel and, on a sample, the oracle."""
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


def gpu_trace(w, ws, scheme=(1, -1, -1), max_ops=4096, budget=0, idx=None):
    store = xd.ReadStore.from_workload(w)
    try:
        pairs, seeds, _ = xd.workload_tensors(w, "cuda")
        if idx is not None:
            sel = torch.from_numpy(np.asarray(idx, np.int64)).cuda()
            pairs, seeds = pairs[sel].contiguous(), seeds[sel].contiguous()
        wt = torch.from_numpy(np.ascontiguousarray(ws, np.int32)).cuda()
        out = xd.banded_traceback(store, pairs, seeds, w=wt, k=w.k, match=scheme[0],
                                  mismatch=scheme[1], gap=scheme[2], max_ops=max_ops,
                                  trace_budget=budget)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        store.close()


def oracle_trace(w, ws, scheme=(1, -1, -1), idx=None):
    idx = np.arange(w.n_tasks) if idx is None else np.asarray(idx)
    return oracle.banded_trace_batch(w.codes, w.off, w.length, np.stack([w.ra, w.rb], 1)[idx],
                                     np.stack([w.pa, w.pb], 1)[idx], ws, k=w.k, match=scheme[0],
                                     mismatch=scheme[1], gap=scheme[2])


def assert_same(got, ref, label, max_ops=4096):
    n = ref["score"].shape[0]
    need = np.array([r.size for r in ref["ops"]], np.int64)
    # a path longer than max_ops entries is reported, not returned
    ref = dict(ref, status=np.where((ref["status"] == 0) & (need > max_ops),
                                    xd.TASK_OPS_OVERFLOW, ref["status"]))
    for key in ("status", "score"):
        bad = np.nonzero(got[key] != ref[key])[0]
        assert bad.size == 0, "%s %s at %s: gpu %s oracle %s" % (
            label, key, bad[:5], got[key][bad[:5]], ref[key][bad[:5]])
    for key in ("end", "beg"):
        bad = np.nonzero((got[key].view(np.uint32) != ref[key]).any(1))[0]
        assert bad.size == 0, "%s %s at %s: gpu %s oracle %s" % (
            label, key, bad[:5], got[key][bad[:5]], ref[key][bad[:5]])
    assert np.array_equal(got["cells"].view(np.uint64), ref["cells"]), label
    for t in range(n):
        r = ref["ops"][t]
        assert got["n_ops"][t] == r.size, "%s task %d: %d ops, oracle %d" % (
            label, t, got["n_ops"][t], r.size)
        if r.size <= max_ops:
            g = got["ops"][t, :r.size].view(np.uint32)
            assert np.array_equal(g, r), "%s task %d: path differs" % (label, t)


@pytest.mark.parametrize("wdt", [0, 8, 32, 48])
def test_trace_c2_small(wdt):
    w = synth.config("c2-small")
    ws = np.full(w.n_tasks, wdt, np.int32)
    assert_same(gpu_trace(w, ws, max_ops=16384), oracle_trace(w, ws), "w=%d" % wdt,
                max_ops=16384)


def edge_workload():
    rng = np.random.default_rng(8)
    A = rand_codes(rng, 3000)
    B = mutate_codes(rng, A, 0.15)
    C = rand_codes(rng, 2000)
    S = rand_codes(rng, 40)
    reads = [A, B, C, S, A[:17].copy()]
    tasks = [(0, 1, 1500, 1480, 0), (0, 1, 0, 0, 0), (0, 1, 2983, 2900, 0),
             (0, 2, 100, 1900, 0), (2, 0, 1900, 100, 0),
             (0, 3, 5, 20, 0), (3, 0, 20, 5, 0), (4, 0, 0, 0, 0), (0, 4, 2983, 0, 0),
             (0, 1, 10, 10, 0), (0, 9, 1, 1, 0), (0, 1, 2990, 5, 0)]
    ws = np.array([24, 48, 48, 48, 48, 10, 10, 5, 48, 49, 8, 8], np.int32)
    return workload_from(reads, tasks), ws


def test_trace_edges_and_statuses():
    w, ws = edge_workload()
    ref = oracle_trace(w, ws)
    assert ref["status"][9] == oracle.TASK_BAD_X and ref["status"][10] == oracle.TASK_BAD_READ
    assert_same(gpu_trace(w, ws), ref, "edges")


@pytest.mark.parametrize("a,b,wdt,scheme,cig", [
    ("ACGTTACG", "ACGTACG", 3, (1, -1, -1), "3M1D4M"),    # diagonal before (i-1, j)
    ("ACGTACG", "ACGTTACG", 3, (1, -1, -1), "3M1I4M"),    # diagonal before (i, j-1)
    ("ACGTAGGGG", "ACGTCGGGG", 4, (1, -3, -1), "4M1I1D4M"),  # (i-1, j) before (i, j-1)
])
def test_trace_tie_rule_cases(a, b, wdt, scheme, cig):
    # the oracle's hand-worked tie cases, on the GPU (seed (0, 0): band around
    # the main diagonal)
    code = {c: q for q, c in enumerate("ACGT")}
    reads = [np.array([code[c] for c in r], np.uint8) for r in (a, b)]
    w = workload_from(reads, [(0, 1, 0, 0, 0)], k=1)
    ws = np.array([wdt], np.int32)
    got = gpu_trace(w, ws, scheme)
    ref = oracle_trace(w, ws, scheme)
    assert_same(got, ref, "tie case %s/%s" % (a, b))
    ops = got["ops"][0, :got["n_ops"][0]].view(np.uint32)
    assert "".join("%d%s" % (e >> 2, "MID"[e & 3]) for e in ops) == cig


@pytest.mark.parametrize("scheme", [(2, -3, -2), (5, -4, -7)])
def test_trace_scoring(scheme):
    w = synth.config("c1-small")
    ws = np.full(w.n_tasks, 20, np.int32)
    assert_same(gpu_trace(w, ws, scheme), oracle_trace(w, ws, scheme), "scheme %s" % (scheme,))


def test_trace_budget_sub_batches():
    # a budget below one task runs every task alone; a middling one mixes
    w = synth.config("c2-small")
    ws = np.full(w.n_tasks, 32, np.int32)
    full = gpu_trace(w, ws)
    for budget in (1, 200_000):
        part = gpu_trace(w, ws, budget=budget)
        for key in full:
            assert np.array_equal(full[key], part[key]), (budget, key)


def test_trace_op_capacity():
    w = synth.config("c2-small")
    ws = np.full(w.n_tasks, 16, np.int32)
    ref = oracle_trace(w, ws)
    cap = 2000  # whole-read paths here need 300..7,000 run-length entries
    got = gpu_trace(w, ws, max_ops=cap)
    need = np.array([r.size for r in ref["ops"]])
    assert (need > cap).any() and (need <= cap).any()
    assert np.array_equal(got["n_ops"], need)
    assert np.array_equal(got["status"] == xd.TASK_OPS_OVERFLOW, need > cap)
    ok = np.nonzero(need <= cap)[0]
    for t in ok:
        assert np.array_equal(got["ops"][t, :need[t]].view(np.uint32), ref["ops"][t])


def test_trace_c2_full_batch():
    # 100,000 whole-read tasks: score, end and cells equal the untraced kernel
    # on every task; begin and path equal the oracle on a sample
    w = synth.config("c2")
    ws = np.full(w.n_tasks, 32, np.int32)
    got = gpu_trace(w, ws, max_ops=4096)
    store = xd.ReadStore.from_workload(w)
    pairs, seeds, _ = xd.workload_tensors(w, "cuda")
    plain = xd.banded_batch(store, pairs, seeds, w_scalar=32, k=w.k)
    torch.cuda.synchronize()
    plain = {k: v.cpu().numpy() for k, v in plain.items()}
    store.close()
    for key in ("score", "end", "cells"):
        assert np.array_equal(got[key], plain[key]), key
    assert (plain["status"] == 0).all()
    over = got["n_ops"] > 4096
    assert np.array_equal(got["status"], np.where(over, xd.TASK_OPS_OVERFLOW, 0))
    idx = np.linspace(0, w.n_tasks - 1, 60).astype(np.int64)
    ref = oracle_trace(w, ws[idx], idx=idx)
    sub = {k: v[idx] for k, v in got.items()}
    assert_same(sub, ref, "c2 sample")
