"""Small statistics helpers shared by the statistical tests (no method arithmetic)."""
import numpy as np


def block_mean_se(values, nblocks=20):
    v = np.asarray(values, dtype=np.float64)
    n = len(v) // nblocks
    if n == 0:
        raise ValueError("series too short")
    b = v[: n * nblocks].reshape(nblocks, n).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(nblocks)


def mean_se(values):
    v = np.asarray(values, dtype=np.float64)
    return v.mean(), v.std(ddof=1) / np.sqrt(len(v))
