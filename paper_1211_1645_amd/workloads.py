"""Seeded synthetic workloads (inputs only; no sampler arithmetic).

The paper's systems are generated from a lattice start and a seed; these
helpers fix the parameter draws used by the benchmark and the tests.
"""
import numpy as np

BATCH_SIDES = (64, 96, 128, 192, 256)


def batch_boxes(nbox=64, seed=0, eta_lo=0.69, eta_hi=0.73, sides=BATCH_SIDES):
    """Independent boxes of uneven size and density: N = side^2 with side
    drawn uniformly from `sides`, eta uniform in [eta_lo, eta_hi], Philox key
    seed + b for box b."""
    rng = np.random.default_rng(seed)
    side = rng.choice(np.asarray(sides), size=nbox)
    eta = rng.uniform(eta_lo, eta_hi, size=nbox)
    N = (side.astype(np.int64) ** 2).astype(np.uint32)
    seeds = (np.uint64(seed) + np.arange(nbox, dtype=np.uint64)).astype(np.uint64)
    return N, eta, seeds
