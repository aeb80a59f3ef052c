"""Host-side checks of the tail-imbalance statistics (paper section 9's
max/avg load imbalance, taken per compute unit from per-wave intervals)."""
import numpy as np

from paper_2001_10049_amd import imbalance as im


def _rec(rows):
    """rows: (t0, t1, tag, xcc, hw_id, items) -> encoded (n, 3) uint64."""
    out = np.zeros((len(rows), 3), np.uint64)
    for i, (t0, t1, tag, xcc, hw, items) in enumerate(rows):
        out[i, 0] = t0
        out[i, 1] = t1
        out[i, 2] = (tag << 56) | (xcc << 48) | (hw << 32) | items
    return out


def test_union_length():
    s = np.array([5.0, 0.0, 1.0, 2.5])
    e = np.array([6.0, 2.0, 3.0, 2.75])
    assert im.union_length(s, e) == 4.0
    assert im.union_length(np.array([1.0]), np.array([4.0])) == 3.0


def test_decode_fields():
    d = im.decode(_rec([(100, 300, 0x20, 7, (3 << 8) | (1 << 4), 12)]))
    assert d["tag"][0] == 0x20 and d["items"][0] == 12
    assert d["cu"][0] == (7 << 8) | 3
    assert np.isclose(d["t1"][0] - d["t0"][0], 2.0)  # 200 ticks of 100 MHz = 2 us


def test_kernel_stats_persistent():
    # two CUs, persistent tier: CU 0's waves busy 0..100 and 0..40 ticks,
    # CU 1's busy 0..50; the first wave with work leaves at tick 40
    rows = [(0, 100, 0x20, 0, 0 << 8, 5), (0, 40, 0x20, 0, 0 << 8, 2),
            (0, 50, 0x20, 0, 1 << 8, 3)]
    st = im.kernel_stats(im.decode(_rec(rows)), 0x20)
    assert st["cus"] == 2 and st["waves"] == 3 and st["items"] == 10
    assert abs(st["cu_max_avg"] - (100 / 75)) < 1e-3
    assert abs(st["drain_share"] - (0.6)) < 1e-3
    # 3 waves up to 40, 2 to 50, 1 to 100: busy 190 of 3 x 100
    assert abs(st["occ"] - (190 / 300)) < 1e-3
    assert np.isclose(st["partial_share"], 0.5)  # 1 of 3 waves from 50 to 100
    assert st["peak_waves"] == 3


def test_kernel_stats_per_item_grid():
    # one-wave-per-item grid: the work runs out when the last wave starts
    rows = [(0, 10, 0x01, 0, 0, 1), (10, 20, 0x01, 0, 0, 1), (5, 80, 0x01, 0, 1 << 8, 1),
            (20, 30, 0x01, 0, 0, 1)]
    st = im.kernel_stats(im.decode(_rec(rows)), 0x01)
    assert abs(st["drain_share"] - (60 / 80)) < 1e-3
    assert abs(st["cu_max_avg"] - (75 / ((30 + 75) / 2))) < 1e-3
