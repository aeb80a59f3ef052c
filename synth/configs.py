"""Named workload recipes.

Each recipe stands in for a workload shaped like the paper's E. coli runs
(section 5) or scaled from it.  Scoring for every recipe is +1/-1/-1
(match/mismatch/gap, linear gaps) with k = 17.

c1  1,000 independent pairs from a 200 kbp genome, read lengths uniform
    2-5 kbp, 5/5/5 % sub/ins/del, template overlap >= 1 kbp, one true seed,
    X = 7.
c2  4.6 Mbp genome at 30x, lengths log-normal (mean 10 kbp, sd 5 kbp,
    clipped 1-50 kbp), 5/5/5 % errors; 100,000 distinct read pairs with
    template overlap >= 1 kbp, one uniformly chosen true seed each; X = 25.
c3  the c2 read set; 2,000,000 (pair, seed) tasks drawn from every pair's
    true seeds kept >= k apart (the paper's "all seeds separated by at least
    k" option); X uniform per task over {7, 25, 50}.
c4  100 Mbp genome = 90 Mbp uniform + 2,000 exact copies of 200 random
    5 kbp segments; 30x, lengths log-normal (12 kbp, sd 6 kbp, clipped
    1-60 kbp), 4/4/4 % errors; 20,000,000 (pair, seed) tasks, 10 % of them
    from reads over two different copies of one segment; X = 25.
c5  serving store: 4.6 Mbp at 30x, lengths log-normal (10 kbp, sd 5 kbp,
    clipped 1-100 kbp); a pool of true (pair, seed) tasks the request
    generator draws from; X per request from {7, 25}.

Suffix "-small" variants keep the shapes at sizes the oracle finishes in
seconds.
"""
from __future__ import annotations

CONFIGS = {
    "c1": dict(seed=1, genome_len=200_000, mode=0, len_dist=0, len_min=2_000, len_max=5_000,
               n_tasks=1_000, x=(7,)),
    "c2": dict(seed=2, genome_len=4_600_000, mode=1, depth=30.0, len_dist=1,
               len_mean=10_000.0, len_sd=5_000.0, len_min=1_000, len_max=50_000,
               n_tasks=100_000, seeds_per_pair=0, x=(25,)),
    "c3": dict(seed=2, genome_len=4_600_000, mode=1, depth=30.0, len_dist=1,
               len_mean=10_000.0, len_sd=5_000.0, len_min=1_000, len_max=50_000,
               n_tasks=2_000_000, seeds_per_pair=1, x=(7, 25, 50)),
    "c4": dict(seed=4, genome_len=90_000_000, n_rep_src=200, rep_len=5_000, n_rep_copies=2_000,
               mode=1, depth=30.0, len_dist=1, len_mean=12_000.0, len_sd=6_000.0,
               len_min=1_000, len_max=60_000, p_sub=0.04, p_ins=0.04, p_del=0.04,
               n_tasks=20_000_000, seeds_per_pair=1, x=(25,), spurious_frac=0.1),
    "c5": dict(seed=5, genome_len=4_600_000, mode=1, depth=30.0, len_dist=1,
               len_mean=10_000.0, len_sd=5_000.0, len_min=1_000, len_max=100_000,
               n_tasks=2_000_000, seeds_per_pair=1, x=(7, 25)),
    # small shapes for CPU tests and quick GPU parity
    "c1-small": dict(seed=11, genome_len=200_000, mode=0, len_dist=0, len_min=2_000,
                     len_max=5_000, n_tasks=64, x=(7,)),
    "c2-small": dict(seed=12, genome_len=150_000, mode=1, depth=30.0, len_dist=1,
                     len_mean=10_000.0, len_sd=5_000.0, len_min=1_000, len_max=50_000,
                     n_tasks=300, seeds_per_pair=0, x=(25,)),
    "c3-small": dict(seed=13, genome_len=150_000, mode=1, depth=30.0, len_dist=1,
                     len_mean=10_000.0, len_sd=5_000.0, len_min=1_000, len_max=50_000,
                     n_tasks=3_000, seeds_per_pair=1, x=(7, 25, 50)),
    "c5-small": dict(seed=15, genome_len=300_000, mode=1, depth=30.0, len_dist=1,
                     len_mean=10_000.0, len_sd=5_000.0, len_min=1_000, len_max=100_000,
                     n_tasks=6_000, seeds_per_pair=1, x=(7, 25)),
    "c4-small": dict(seed=14, genome_len=900_000, n_rep_src=4, rep_len=5_000, n_rep_copies=20,
                     mode=1, depth=30.0, len_dist=1, len_mean=12_000.0, len_sd=6_000.0,
                     len_min=1_000, len_max=60_000, p_sub=0.04, p_ins=0.04, p_del=0.04,
                     n_tasks=2_000, seeds_per_pair=1, x=(25,), spurious_frac=0.1),
}


def config(name: str, **override):
    """Generate the named workload (overrides replace recipe fields)."""
    from . import make
    if name not in CONFIGS:
        raise KeyError("unknown workload %r (have %s)" % (name, sorted(CONFIGS)))
    p = dict(CONFIGS[name])
    p.update(override)
    return make(name=name, **p)
