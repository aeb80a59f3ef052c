"""Host-side checks of the autotuner's search space and calibration slice."""
import re

import numpy as np

from paper_2001_10049_amd import tune


class _W:
    def __init__(self, xs, n, lengths=(10000,)):
        self.x = np.asarray(xs, np.int32)
        self.n_tasks = n
        self.length = np.asarray(lengths, np.uint32)


def _firsts(t, xs):
    return tuple(0 if x <= t["x_tier1"] else 1 if x <= t["x_tier2"] else 2 for x in xs)


def test_candidates_cover_each_first_window_assignment_once():
    for xs in ([25], [7, 25, 50], [7]):
        w = _W(xs, 1000)
        cands = list(tune.candidates(w))
        keys = [(t["waves_per_cu"], t["group_steps"], t["order"], _firsts(t, sorted(set(xs))))
                for t in cands]
        assert len(keys) == len(set(keys))
        assert all(t["x_tier1"] <= t["x_tier2"] for t in cands)
        # every (waves, group, order) setting appears with every reachable assignment
        per = {}
        for k in keys:
            per.setdefault(k[:3], set()).add(k[3])
        assert len(set(map(frozenset, per.values()))) == 1
    # X = 25 can start in the 64- or the 128-cell window; 7, 25, 50 in three ways
    assert {k for k in (_firsts(t, [25]) for t in tune.candidates(_W([25], 1)))} == {(0,), (1,)}
    got = {_firsts(t, [7, 25, 50]) for t in tune.candidates(_W([7, 25, 50], 1))}
    assert got == {(0, 1, 1), (0, 0, 1), (0, 0, 0)}


def test_calibration_slice_is_one_percent_repeated_to_full_scale():
    assert tune.slice_size(_W([25], 100_000)) == 2_000
    assert tune.slice_size(_W([25], 2_000_000)) == 20_000
    assert tune.slice_size(_W([25], 20_000_000)) == 200_000
    assert tune.slice_size(_W([25], 500)) == 500
    for n in (500, 100_000, 2_000_000, 20_000_000):
        idx = tune.calibration_tasks(_W([25], n), seed=3)
        k = tune.slice_size(_W([25], n))
        assert idx.size >= tune.LAUNCH_MIN and idx.size % k == 0
        uniq = np.unique(idx)
        assert uniq.size == k and uniq.min() >= 0 and uniq.max() < n
        # every sampled task appears equally often
        assert (np.bincount(idx)[uniq] == idx.size // k).all()


def test_signature_and_key_without_gpu():
    w = _W([25, 7, 25], 10, lengths=[9000, 11000, 10500])
    assert tune.signature(w) == "x7-25_L10k"
    key = tune.device_key()  # "unknown" without a GPU
    assert key == "unknown" or re.fullmatch(r"gfx[0-9a-f]+_[0-9]+cu", key), key
