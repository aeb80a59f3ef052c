"""GPU parity for multi-seed pair alignment (xd_align_pairs) against the
oracle (oracle/pairs.py): seed selection under the paper's options, the
reverse strand, and the best-per-pair rule."""
import numpy as np
import pytest

import synth
from oracle import pairs as op

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2001_10049_amd as xd  # noqa: E402


def multiseed_pairs(n_pairs=150, seed=31):
    """Pairs from c3-small with every true seed kept >= k apart, lists sorted by
    pa.  Odd pairs are reverse-strand twins: B is stored reverse-complemented
    (an extra read), so aligning it reverse-complemented must reproduce the
    forward pair exactly, in the same coordinates."""
    w = synth.config("c3-small", n_tasks=10 ** 7)   # every candidate (pair, seed) task
    a = np.minimum(w.ra, w.rb)
    b = np.maximum(w.ra, w.rb)
    flip = w.ra > w.rb
    pa = np.where(flip, w.pb, w.pa)
    pb = np.where(flip, w.pa, w.pb)
    keys = a.astype(np.uint64) << 32 | b.astype(np.uint64)
    uk = np.unique(keys)
    rng = np.random.default_rng(seed)
    chosen = rng.choice(uk, min(n_pairs, uk.size), replace=False)
    codes, off, length = [w.codes], list(w.off), list(w.length)
    total = int(w.codes.size)
    pairs, rc, lists, xs, fwd_b = [], [], [], [], []
    for q, key in enumerate(chosen):
        sel = np.nonzero(keys == key)[0]
        order = np.lexsort((pb[sel], pa[sel]))
        ra, rb = int(a[sel[0]]), int(b[sel[0]])
        lists.append(np.stack([pa[sel][order], pb[sel][order]], 1))
        xs.append(int(rng.choice([7, 25, 50])))
        fwd_b.append(rb)
        if q % 2:
            seq = w.codes[int(w.off[rb]):int(w.off[rb]) + int(w.length[rb])]
            codes.append(op.revcomp(seq))
            off.append(total)
            length.append(int(w.length[rb]))
            total += int(w.length[rb])
            pairs.append((ra, len(length) - 1))
            rc.append(1)
        else:
            pairs.append((ra, rb))
            rc.append(0)
    # one pair with an empty list
    pairs.append(pairs[0])
    rc.append(0)
    lists.append(np.zeros((0, 2), np.uint32))
    xs.append(25)
    fwd_b.append(pairs[0][1])
    seed_off = np.concatenate([[0], np.cumsum([len(l) for l in lists])]).astype(np.uint64)
    return dict(codes=np.concatenate(codes), off=np.array(off, np.uint64),
                length=np.array(length, np.uint32), pairs=np.array(pairs, np.uint32),
                rc=np.array(rc, np.uint8), seed_off=seed_off,
                seeds=np.concatenate(lists).astype(np.uint32), x=np.array(xs, np.int32),
                fwd_b=np.array(fwd_b, np.uint32))


def gpu_pairs(d, store, rc, b_col, min_dist, max_seeds):
    pairs = np.stack([d["pairs"][:, 0], b_col], 1).astype(np.uint32)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()  # noqa: E731
    out = xd.align_pairs(store, t(pairs, np.int32), t(d["seed_off"], np.int64),
                         t(d["seeds"], np.int32), rc=t(rc, np.uint8), x=t(d["x"], np.int32),
                         min_dist=min_dist, max_seeds=max_seeds, k=17)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def same(got, ref, label):
    for key in ("status", "score", "n_kept"):
        g, r = got[key].astype(np.int64), ref[key].astype(np.int64)
        bad = np.nonzero(g != r)[0]
        assert bad.size == 0, "%s %s differs at %s: %s vs %s" % (label, key, bad[:5], g[bad[:5]],
                                                                r[bad[:5]])
    u32 = lambda a: np.ascontiguousarray(a).view(np.uint32)  # noqa: E731
    assert np.array_equal(u32(got["seed_idx"]), u32(ref["seed_idx"])), label
    assert np.array_equal(u32(got["beg"]), u32(ref["beg"])), label
    assert np.array_equal(u32(got["end"]), u32(ref["end"])), label
    assert np.array_equal(np.ascontiguousarray(got["cells"]).view(np.uint64),
                          np.ascontiguousarray(ref["cells"]).view(np.uint64)), label


@pytest.fixture(scope="module")
def data():
    d = multiseed_pairs()
    store = xd.ReadStore(d["codes"], d["off"], d["length"])
    yield d, store
    store.close()


@pytest.mark.parametrize("min_dist,max_seeds", [(17, 0), (1000, 0), (17, 1), (0, 5)])
def test_pairs_match_oracle(data, min_dist, max_seeds):
    d, store = data
    print("pairs", min_dist, max_seeds, len(d["pairs"]), "pairs", len(d["seeds"]), "seeds",
          flush=True)
    got = gpu_pairs(d, store, d["rc"], d["pairs"][:, 1], min_dist, max_seeds)
    ref = op.align_pairs(d["codes"], d["off"], d["length"], d["pairs"], d["seed_off"],
                         d["seeds"], rc=d["rc"], x=d["x"], min_dist=min_dist,
                         max_seeds=max_seeds)
    same(got, ref, "pairs %d/%d" % (min_dist, max_seeds))
    assert (got["status"][:-1] == 0).all() and got["status"][-1] == xd.TASK_NO_SEED


def test_reverse_strand_twins_equal_forward(data):
    d, store = data
    twin = gpu_pairs(d, store, d["rc"], d["pairs"][:, 1], 17, 0)
    fwd = gpu_pairs(d, store, np.zeros_like(d["rc"]), d["fwd_b"], 17, 0)
    assert d["rc"].sum() > 50
    same(twin, fwd, "twins")
