"""Checks on the seeded workload generator (no GPU)."""
import numpy as np

import synth


def test_deterministic():
    a = synth.config("c1-small")
    b = synth.config("c1-small")
    for f in ("codes", "off", "length", "ra", "rb", "pa", "pb", "x"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_seeds_are_exact_shared_kmers():
    for name in ("c1-small", "c2-small", "c3-small", "c4-small"):
        w = synth.config(name)
        assert w.n_tasks > 0
        for t in range(w.n_tasks):
            A, B = w.read(int(w.ra[t])), w.read(int(w.rb[t]))
            assert np.array_equal(A[w.pa[t]:w.pa[t] + w.k], B[w.pb[t]:w.pb[t] + w.k]), (name, t)


def test_pair_mode_shape():
    w = synth.config("c1-small")
    assert w.n_reads == 2 * w.n_tasks
    assert (w.length >= 2000).all() and (w.length <= 5000).all()
    assert (w.ovl >= 1000).all()
    assert set(np.unique(w.x)) == {7}


def test_coverage_mode_shape():
    w = synth.config("c2-small", keep_genome=True)
    G = w.genome.size
    assert abs(int(w.length.sum()) / G - 30.0) < 1.0          # 30x depth
    assert 8000 < w.length.mean() < 12000                      # log-normal mean 10 kbp
    assert w.length.min() >= 1000 and w.length.max() <= 50000
    # 5 % insertions and 5 % deletions balance: read length ~ template span
    span = (w.tspan[:, 1] - w.tspan[:, 0]).astype(np.float64)
    assert abs(w.length.sum() / span.sum() - 1.0) < 0.01
    assert (w.ovl >= 1000).all()
    # distinct pairs in one-seed mode
    pairs = set(zip(np.minimum(w.ra, w.rb).tolist(), np.maximum(w.ra, w.rb).tolist()))
    assert len(pairs) == w.n_tasks


def test_substitution_rate_on_template():
    # outside indels the read copies its template; count mismatches between
    # each read's first bases and the genome, up to the first indel-free run
    w = synth.config("c2-small", keep_genome=True)
    # a cheap estimate: the fraction of seeds' neighbourhood is not testable
    # without alignment, so check the base composition instead (uniform ACGT)
    counts = np.bincount(w.codes, minlength=4) / w.codes.size
    assert np.all(np.abs(counts - 0.25) < 0.01)


def test_mixed_x_and_spurious():
    w = synth.config("c3-small")
    assert set(np.unique(w.x)) <= {7, 25, 50} and len(np.unique(w.x)) == 3
    w4 = synth.config("c4-small")
    frac = w4.spurious.mean()
    assert 0.05 < frac < 0.15
    assert (w4.ovl[w4.spurious == 1] == 0).all()
