"""The learned proposal's lattice law and Metropolis-Hastings sweep on the
GPU against the oracle: ln P(D) element by element, the draws element by
element and against the law (chi-square at the lattice scale), the learned
sweep bit for bit (with the plain step only, and with a fixed mixture),
the recording sweep's trajectory and moves, and Adam."""
import math

import numpy as np
import pytest
from scipy.stats import chi2

from oracle import orc
from oracle.orc import OracleBox, Q
from tests import inputs

pytestmark = pytest.mark.gpu


def _one_component(mu_x, mu_y, a_x, a_y):
    out = np.zeros(20, np.float32)
    out[5:20:5] = -1e4
    out[1], out[2], out[3], out[4] = mu_x, mu_y, a_x, a_y
    return out


def test_lattice_logp_matches_oracle(gpu_lib):
    rng = np.random.default_rng(5)
    outs, D = [], []
    for seed in range(40):
        out = inputs.mlp_outputs(seed).astype(np.float32)
        for _ in range(25):
            k = rng.integers(4)
            kind = rng.integers(4)
            if kind == 0:    # near a component mean
                c = np.array([out[5 * k + 1], out[5 * k + 2]]) + \
                    np.exp(out[5 * k + 3: 5 * k + 5]) * rng.normal(size=2) * 2
                d = np.rint(c / Q)
            elif kind == 1:  # a point of the plain step
                d = 26 * (2 * rng.integers(-8192, 8192, 2) + 1)
            elif kind == 2:  # anywhere within reach
                d = rng.integers(-(2 ** 22) + 1, 2 ** 22, 2)
            else:            # the edges of the Gaussian part's support
                d = np.array([rng.choice([-1, 1]) * (2 ** 22 - 1 + rng.integers(2)),
                              rng.integers(-1000, 1000)])
            outs.append(out)
            D.append(d)
    outs = np.array(outs, np.float32)
    D = np.array(D, np.int64)
    for eps in (0.0, 0.1, 1.0):
        got = gpu_lib.learned_logp(outs, D, 26, eps)
        ref = np.array([orc.learned_logp(o.astype(np.float64), d[0], d[1], 26, eps)
                        for o, d in zip(outs, D)])
        fin = ref > -700
        assert fin.sum() > (200 if eps == 1.0 else 800)
        assert np.all(np.abs(got[fin] - ref[fin]) <= 1e-11 * np.maximum(1, np.abs(ref[fin]))), eps
        # below 1e-300 the device's linear-space probability may round to 0
        assert np.all((got[~fin] < -690) | np.isneginf(got[~fin]))


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_lattice_draws_match_oracle(gpu_lib, eps):
    """Same words, same draws: every displacement equal (up to a double
    rounding tie, below 1e-6 of the draws) and every ln P within 1e-11."""
    n = 1_000_000
    for seed in (3, 4):
        out = inputs.mlp_outputs(seed).astype(np.float32)
        D, dr, lp = gpu_lib.learned_propose(out, 26, eps, 17 + seed, n)
        Do, dro, lpo = orc.learned_proposals(out.astype(np.float64), 26, eps, 17 + seed, n)
        assert np.array_equal(dr, dro)
        diff = np.any(D != Do, axis=1)
        assert diff.sum() <= 1, np.nonzero(diff)
        assert np.all(np.abs(D[diff] - Do[diff]) <= 1)
        same = dr & ~diff
        assert np.all(np.abs(lp[same] - lpo[same]) <= 1e-11 * np.abs(lpo[same]))


def test_lattice_draws_follow_the_law_at_the_lattice_scale(gpu_lib):
    """4e6 draws of a 300 q component: counts on every lattice cell within
    28 q of the mean against n P(D) from the oracle (chi-square)."""
    s = 300 * Q
    out = _one_component(0.01 + 0.3 * Q, -0.02 + 0.6 * Q, math.log(s), math.log(s))
    n = 4_000_000
    D, drawn, _ = gpu_lib.learned_propose(out, 26, 0.0, 99, n)
    assert drawn.all()
    c = np.rint(out[1:3].astype(np.float64) / Q).astype(np.int64)
    R = 28
    inwin = (np.abs(D[:, 0] - c[0]) <= R) & (np.abs(D[:, 1] - c[1]) <= R)
    idx = (D[inwin, 0] - c[0] + R) * (2 * R + 1) + (D[inwin, 1] - c[1] + R)
    counts = np.bincount(idx, minlength=(2 * R + 1) ** 2)
    o64 = out.astype(np.float64)
    expect = np.array([n * math.exp(orc.learned_logp(o64, c[0] + i - R, c[1] + j - R, 26, 0.0))
                       for i in range(2 * R + 1) for j in range(2 * R + 1)])
    x2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2.sf(x2, len(counts)) > 1e-4, x2


def test_lattice_draws_resolve_the_lattice_near_a_wide_mean(gpu_lib):
    """Width 1 sigma, mean on a lattice point: among draws within 0.02 sigma
    Dx^2 + Dy^2 modulo 2^21 is uniform (a 24-bit draw fails this, see the
    oracle pins)."""
    out = _one_component(0.0, 0.0, 0.0, 0.0)
    D, drawn, _ = gpu_lib.learned_propose(out, 26, 0.0, 5, 8_000_000)
    D = D[drawn].astype(np.int64)
    near = D[(D ** 2).sum(1) < (0.02 / Q) ** 2]
    r2 = (near ** 2).sum(1)
    h = np.bincount(((r2 % 2 ** 21) * 16) >> 21, minlength=16)
    e = len(near) / 16
    assert len(near) > 1000
    assert chi2.sf(((h - e) ** 2 / e).sum(), 15) > 1e-4, h


def _pair(gpu_lib, N, eta, seed, lattice, step_m, n_trial=1):
    g = gpu_lib.Box(N, eta, seed=seed, step_m=step_m, n_trial=n_trial, cell_min=3.0,
                    lattice=lattice, schedule="simple")
    o = OracleBox(N, eta, seed=seed, cell_min=3.0, lattice=1 if lattice == "triangular" else 0,
                  step_m=step_m, n_trial=n_trial)
    return g, o


def _same_cells(g, o):
    for a, b in zip(g.cells(), o.cells()):
        assert np.array_equal(a, b)


def test_learned_sweep_with_plain_step_only_is_the_plain_sweep(gpu_lib):
    """eps = 1: the learned sweep is the plain sweep word for word, on the
    GPU as in the oracle, whatever the network."""
    L = gpu_lib.Learner(seed=1, capacity=16)
    L.set_params(inputs.mlp_params(8))
    g, o = _pair(gpu_lib, 4096, 0.70, 12, "triangular", 40)
    p = gpu_lib.Box(4096, 0.70, seed=12, step_m=40, cell_min=3.0, schedule="simple")
    t, a = gpu_lib.sweep_learned(g, L, 10, eps=1.0, counts=True)
    tp, ap = p.sweep(10, counts=True)
    o.sweep(10)
    assert (t, a) == (tp, ap) == (o.info()["trials"], o.info()["accepts"])
    _same_cells(g, o)
    _same_cells(p, o)


@pytest.mark.parametrize("N,eta,lattice,n_trial,sweeps", [
    (256, 0.60, "square", 1, 30), (256, 0.60, "square", 3, 10), (4096, 0.70, "triangular", 1, 12)])
def test_learned_sweep_fixed_mixture_bit_exact(gpu_lib, N, eta, lattice, n_trial, sweeps):
    """A network whose output does not depend on the features (last layer
    zero, bias = a mixture) makes the learned sweep a deterministic function
    of the words on both sides: the GPU's bf16 network, the double-precision
    draws, the lattice law and the acceptance reproduce the oracle's
    trajectory bit for bit."""
    out = inputs.mlp_outputs(21).astype(np.float32)
    p = inputs.fixed_output_params(4, out)
    L = gpu_lib.Learner(seed=1, capacity=16)
    L.set_params(p)
    g, o = _pair(gpu_lib, N, eta, 33, lattice, 30, n_trial)
    t, a = gpu_lib.sweep_learned(g, L, sweeps, eps=0.3, counts=True)
    o.sweep_learned(p.astype(np.float64), 0.3, sweeps)
    assert (t, a) == (o.info()["trials"], o.info()["accepts"])
    assert 0.05 * t < a < 0.95 * t
    _same_cells(g, o)
    assert g.validate() == (0, 0)


def test_collect_records_the_oracles_moves(gpu_lib):
    """The recording sweep follows the plain trajectory, and the recorded
    (features at the old position, displacement) rows are the oracle's, as
    a multiset (the device records in the order of its atomic counter)."""
    g, o = _pair(gpu_lib, 4096, 0.70, 7, "triangular", 40)
    L = gpu_lib.Learner(seed=2, capacity=1 << 16)
    n = L.collect(g, 6)
    Fo, Do, tot = o.sweep_collect(6, 1 << 16)
    assert n == tot == o.info()["accepts"] and n > 1000
    _same_cells(g, o)
    F, D = L.moves()
    rows = np.concatenate([F, D], 1)
    rows_o = np.concatenate([Fo, Do], 1)
    key = lambda r: r[np.lexsort(r.T[::-1])]
    assert np.array_equal(key(rows), key(rows_o))


def test_adam_matches_oracle(gpu_lib):
    """Ten Adam steps with given gradients: the fp32 master weights follow
    the oracle's fp64 Adam within fp32 rounding."""
    rng = np.random.default_rng(3)
    p0 = inputs.mlp_params(5).astype(np.float32)
    L = gpu_lib.Learner(seed=1, capacity=16)
    L.set_params(p0)
    p = p0.astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    for t in range(1, 11):
        grad = (rng.standard_normal(p.size) * 10.0 ** rng.uniform(-4, 0, p.size)).astype(np.float32)
        L.adam_step(grad, 1e-3)
        orc.adam(p, m, v, grad.astype(np.float64), 1e-3, t)
    got = L.params().astype(np.float64)
    assert np.abs(got - p).max() < 2e-6, np.abs(got - p).max()
    assert np.abs(got - p0).max() > 5e-3  # the steps did move the weights


def test_learned_graph_replays_match_direct_launches(gpu_lib):
    """Runs of learned sweeps replay captured graphs of 8 sweeps; with graphs
    off every sweep is launched directly.  Both give the same trajectory and
    counts, from an odd start (direct sweeps until the lists are back in
    their first buffer), across a change of eps (a new capture) and a new
    learner."""
    L = gpu_lib.Learner(seed=1, capacity=16)
    L.set_params(inputs.mlp_params(8))
    a = gpu_lib.Box(4096, 0.70, seed=5, step_m=40, cell_min=3.0, schedule="simple")
    b = gpu_lib.Box(4096, 0.70, seed=5, step_m=40, cell_min=3.0, schedule="simple")
    b.set_graphs(0)
    for k, eps in ((1, 0.1), (19, 0.1), (16, 0.3), (8, 0.3)):
        assert (gpu_lib.sweep_learned(a, L, k, eps=eps, counts=True) ==
                gpu_lib.sweep_learned(b, L, k, eps=eps, counts=True))
    L2 = gpu_lib.Learner(seed=2, capacity=16)
    L2.set_params(inputs.mlp_params(9))
    assert (gpu_lib.sweep_learned(a, L2, 24, eps=0.2, counts=True) ==
            gpu_lib.sweep_learned(b, L2, 24, eps=0.2, counts=True))
    for x, y in zip(a.cells(), b.cells()):
        assert np.array_equal(x, y)
    assert a.validate() == (0, 0)


def test_learned_cells_per_wave_do_not_change_the_trajectory(gpu_lib):
    """The learned pass spreads a colour's cells over waves of 16, 32 or 64
    cells; random numbers are keyed by cell and every network row is its own,
    so the trajectory and the counts are the same for each choice (and for
    the automatic one)."""
    L = gpu_lib.Learner(seed=1, capacity=16)
    L.set_params(inputs.mlp_params(8))
    runs = []
    for cells in (0, 16, 32, 64):
        b = gpu_lib.Box(4096, 0.70, seed=9, step_m=40, cell_min=3.0, schedule="simple")
        b.set_learned_cells_per_wave(cells)
        counts = gpu_lib.sweep_learned(b, L, 11, eps=0.2, counts=True)
        runs.append((counts, [c.copy() for c in b.cells()]))
    for counts, cells in runs[1:]:
        assert counts == runs[0][0]
        for x, y in zip(cells, runs[0][1]):
            assert np.array_equal(x, y)
    b = gpu_lib.Box(4096, 0.70, seed=9, step_m=40, cell_min=3.0, schedule="simple")
    with pytest.raises(gpu_lib.MPMCError):
        b.set_learned_cells_per_wave(48)
