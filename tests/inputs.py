"""Seeded random inputs shared by oracle and GPU tests (no method arithmetic)."""
import numpy as np

NPARAM = 7060


def mlp_params(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(NPARAM) * scale
    # output biases: moderate log widths so the mixture is well conditioned
    b3 = NPARAM - 20
    for k in range(4):
        p[b3 + 5 * k + 3] = np.log(0.05) + 0.3 * rng.standard_normal()
        p[b3 + 5 * k + 4] = np.log(0.05) + 0.3 * rng.standard_normal()
    return p


def features(seed, B):
    """Feature rows like real neighbourhoods: 3-11 neighbours within 3 sigma,
    sorted by distance, zero padded."""
    rng = np.random.default_rng(seed)
    F = np.zeros((B, 24))
    for b in range(B):
        n = rng.integers(3, 12)
        r = np.sort(rng.uniform(2.0, 3.0, n))
        phi = rng.uniform(0, 2 * np.pi, n)
        F[b, 0:2 * n:2] = r * np.cos(phi)
        F[b, 1:2 * n:2] = r * np.sin(phi)
    return F


def moves(seed, B, d=0.1):
    rng = np.random.default_rng(seed)
    return rng.uniform(-d, d, size=(B, 2))


def mlp_outputs(seed):
    """A network output vector (20 numbers) shaped like a trained one: logits
    of order 1, means within 0.2 sigma, log widths around ln 0.05."""
    rng = np.random.default_rng(seed)
    out = np.zeros(20)
    for k in range(4):
        out[5 * k] = rng.standard_normal()
        out[5 * k + 1: 5 * k + 3] = rng.uniform(-0.2, 0.2, 2)
        out[5 * k + 3: 5 * k + 5] = np.log(0.05) + 0.5 * rng.standard_normal(2)
    return out.astype(np.float32).astype(np.float64)


def fixed_output_params(seed, out):
    """Network parameters (fp32 values) whose last layer has zero weights, so
    that the output is the bias b3 = out whatever the features: the hidden
    layers are random and still evaluated."""
    p = mlp_params(seed).astype(np.float32)
    b3 = NPARAM - 20
    w3 = b3 - 20 * 64
    p[w3:b3] = 0.0
    p[b3:] = np.asarray(out, np.float32)
    return p
