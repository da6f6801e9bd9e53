"""The learned proposal on the GPU: features bit for bit and the BF16-MFMA
network forward and backward within bf16 tolerance of the fp64 oracle; the
MH-corrected sampler exact on the N = 2 closed form and in agreement with
the plain sampler; training reduces the loss."""
import math

import numpy as np
import pytest

from oracle import orc
from oracle.orc import OracleBox
from tests import inputs
from tests.stats import mean_se

pytestmark = pytest.mark.gpu


def test_features_match_oracle(gpu_lib):
    cfg = dict(N=64 * 64, eta=0.716, seed=2)
    g = gpu_lib.Box(**cfg, step_m=30, cell_min=3.0, schedule="simple")
    o = OracleBox(**cfg, lattice=1, step_m=30, cell_min=3.0)
    g.sweep(25)
    o.sweep(25)
    cnt, tag, x, y = o.cells()
    assert np.array_equal(cnt, g.cells()[0])
    rng = np.random.default_rng(0)
    tags = rng.choice(cfg["N"], 300, replace=False).astype(np.uint32)
    F = gpu_lib.learned_features(g, tags)
    where = {}
    for c in range(len(cnt)):
        for s in range(cnt[c]):
            where[int(tag[c, s])] = (c, s)
    nonzero = 0
    for r, t in enumerate(tags):
        c, s = where[int(t)]
        f, n = o.features(c, int(t), x[c, s], y[c, s])
        assert np.array_equal(F[r], f), (t, F[r], f)
        nonzero += n
    assert nonzero > 300 * 3


def test_forward_matches_oracle(gpu_lib):
    p = inputs.mlp_params(11)
    L = gpu_lib.Learner(seed=0, capacity=16)
    L.set_params(p)
    F = inputs.features(12, 200)
    out = L.forward(F)
    ref = np.array([orc.mlp_forward(p, f) for f in F])
    err = np.abs(out - ref)
    scale = np.abs(ref).max()
    assert err.max() < 0.03 * scale, (err.max(), scale)
    assert np.corrcoef(out.ravel(), ref.ravel())[0, 1] > 0.9995


def test_nll_gradient_matches_oracle(gpu_lib):
    p = inputs.mlp_params(21)
    L = gpu_lib.Learner(seed=0, capacity=16)
    L.set_params(p)
    F = inputs.features(22, 256)
    D = inputs.moves(23, 256)
    loss, g = L.nll_grad(F, D)
    rloss, rg = orc.nll_grad(p, F, D)
    assert abs(loss - rloss) < 0.02 * abs(rloss) + 0.02, (loss, rloss)
    cos = float(g @ rg / (np.linalg.norm(g) * np.linalg.norm(rg)))
    assert cos > 0.999, cos
    assert np.linalg.norm(g - rg) < 0.05 * np.linalg.norm(rg)
    # every parameter block gets its gradient (biases and weights of all layers)
    for a, b in [(0, 1536), (1536, 1600), (1600, 5696), (5696, 5760), (5760, 7040), (7040, 7060)]:
        assert np.linalg.norm(g[a:b]) > 0
        cb = float(g[a:b] @ rg[a:b] / (np.linalg.norm(g[a:b]) * np.linalg.norm(rg[a:b])))
        assert cb > 0.99, (a, b, cb)


def _n2_box(gpu_lib, seed):
    g = gpu_lib.Box(2, 0.04, seed=seed, step_m=200, lattice="none", cell_min=3.0,
                    hist_bins=100, hist_dr=0.01, hist_block=2000)
    X = np.array([int(1.0 / orc.Q), int(7.5 / orc.Q)], np.int64)
    Y = np.array([int(1.5 / orc.Q), int(8.0 / orc.Q)], np.int64)
    g.set_positions_q(X, Y)
    return g


def test_learned_sampler_exact_for_two_disks(gpu_lib):
    """Whatever the network, the MH correction keeps the uniform
    distribution: P* = (4 eta/pi)(1-eta)/(1-2 eta) for N = 2."""
    L = gpu_lib.Learner(seed=5, capacity=16)
    p = inputs.mlp_params(31, scale=0.3)
    L.set_params(p)
    g = _n2_box(gpu_lib, 41)
    for _ in range(40000):
        gpu_lib.sweep_learned(g, L, 2, eps=0.2)
        g.accumulate_contacts()
    eta = g.info()["eta_eff"]
    res = g.measure_pressure()
    exact = 4 * eta / math.pi * (1 - eta) / (1 - 2 * eta)
    assert abs(res["P_star"] - exact) < 3 * res["se"], (res, exact)
    assert g.validate() == (0, 0)


def test_training_reduces_loss_and_learned_matches_plain(gpu_lib, tmp_path):
    """Collect accepted plain moves on a dense liquid, train, then compare
    the pressure of learned and plain runs (same box size, same w >= 3
    grid).  Each sampler is continued from four independently equilibrated
    configurations and the error comes from the scatter between those runs:
    the block error of one run underestimates the true one by a factor of
    two or more at this size, because the pressure decorrelates slowly."""
    cfg = dict(N=32 * 32, eta=0.65)
    box = gpu_lib.Box(**cfg, seed=7, step_m=40, cell_min=3.0, schedule="simple")
    L = gpu_lib.Learner(seed=3, capacity=1 << 18)
    n = L.collect(box, 300)
    assert n > 10000
    l0 = L.train(1, batch=2048, lr=1e-3)
    l1 = L.train(600, batch=2048, lr=1e-3)
    assert l1 < l0 - 0.3, (l0, l1)
    assert L.info()["feature_overflow"] == 0
    Ps = {"plain": [], "learned": []}
    for seed in range(100, 104):
        eq = gpu_lib.Box(**cfg, seed=seed, step_m=40, cell_min=3.0, schedule="simple",
                         hist_bins=20, hist_dr=0.01, hist_block=500)
        eq.sweep(3000)
        start = str(tmp_path / ("equilibrated_%d.ckpt" % seed))
        eq.save(start)
        for mode in ("plain", "learned"):
            b = gpu_lib.Box.load(start, schedule="simple")
            for _ in range(3000):
                if mode == "plain":
                    b.sweep(2)
                else:
                    gpu_lib.sweep_learned(b, L, 2, eps=0.1)
                b.accumulate_contacts()
            Ps[mode].append(b.measure_pressure()["P_star"])
            assert b.validate() == (0, 0)
    p, q = np.array(Ps["plain"]), np.array(Ps["learned"])
    se = math.sqrt(p.var(ddof=1) / len(p) + q.var(ddof=1) / len(q))
    d = q.mean() - p.mean()
    # 4 standard errors: about 1% false alarms with 6 degrees of freedom
    assert abs(d) < 4 * se, (Ps, d, se)
