"""Pins of the oracle's learned proposal (its law on the q lattice, its draws,
its Metropolis-Hastings sweep), of the move-recording sweep, of the overlap
count, the psi field and Adam beyond the first step.

Each check is against something other than the oracle itself: closed forms,
scipy's normal distribution function, the plain oracle sweep (which the
other pins tie to the paper), exact statistics of the draws, the N = 2
closed form, and configurations built by hand.
"""
import math

import numpy as np
import pytest
from scipy.special import ndtr
from scipy.stats import chi2

from oracle import orc
from oracle.orc import OracleBox, Q
from tests import inputs
from tests.stats import block_mean_se, mean_se

LN2 = math.log(2.0)


def _one_component(mu_x, mu_y, a_x, a_y, others=-1e4):
    """A network output with component 0 only (the other logits -1e4)."""
    out = np.zeros(20)
    out[5:20:5] = others
    out[1], out[2], out[3], out[4] = mu_x, mu_y, a_x, a_y
    return out


def _log_cell_mass_ref(D, mu, s):
    """ln of the N(mu, s^2) mass of [(D - 1/2) q, (D + 1/2) q], from scipy's
    normal distribution function (upper tail where it is the smaller)."""
    a = ((D - 0.5) * Q - mu) / s
    b = ((D + 0.5) * Q - mu) / s
    if a > 0:
        return math.log(ndtr(-a) - ndtr(-b))
    return math.log(ndtr(b) - ndtr(a))


# --------------------------------------------------------------------------
# The law P(D)
def test_logp_uniform_branch_limit():
    """eps = 1: the plain trial's step, 2^-14 per axis on the odd multiples of
    m, nothing elsewhere."""
    out = inputs.mlp_outputs(3)
    m = 26
    rng = np.random.default_rng(0)
    for _ in range(200):
        jx, jy = rng.integers(-8192, 8192, 2) * 2 + 1
        assert orc.learned_logp(out, m * jx, m * jy, m, 1.0) == pytest.approx(-28 * LN2, abs=1e-12)
        # even multiples, off-multiples and beyond 2^14 - 1 steps: impossible
        assert orc.learned_logp(out, m * (jx + 1), m * jy, m, 1.0) == -math.inf
        assert orc.learned_logp(out, m * jx + 1, m * jy, m, 1.0) == -math.inf
    assert orc.learned_logp(out, m * 16385, m, m, 1.0) == -math.inf
    assert orc.learned_logp(out, m * 16383, -m * 16383, m, 1.0) == pytest.approx(-28 * LN2)


@pytest.mark.parametrize("s_q", [200.0, 300.0, 3000.0, 1.0e5])
def test_logp_single_gaussian_is_cell_mass(s_q):
    """eps = 0 and one component: P(D) is the Gaussian mass of the lattice
    cell of D, per axis, as scipy's normal distribution function gives it."""
    s = s_q * Q
    mu_x, mu_y = 0.3 * s + 0.37 * Q, -0.8 * s + 0.11 * Q
    out = _one_component(mu_x, mu_y, math.log(s), math.log(s))
    out = out.astype(np.float32).astype(np.float64)  # outputs are fp32 numbers
    mu_x, mu_y, s = out[1], out[2], math.exp(out[3])
    rng = np.random.default_rng(1)
    for _ in range(300):
        ux, uy = rng.normal(size=2) * 2.5
        Dx, Dy = int(round((mu_x + ux * s) / Q)), int(round((mu_y + uy * s) / Q))
        rx, ry = _log_cell_mass_ref(Dx, mu_x, s), _log_cell_mass_ref(Dy, mu_y, s)
        got = orc.learned_logp(out, Dx, Dy, 26, 0.0)
        # the reference is a difference of two distribution values, each
        # within about 1e-16: a relative error of 1e-16 over the cell mass
        tol = 1e-12 + 4e-16 * (math.exp(-rx) + math.exp(-ry))
        assert abs(got - (rx + ry)) < tol, (Dx, Dy, got, rx + ry)


def test_logp_wide_mixture_is_lattice_density():
    """eps = 0, widths >> q: P(D) = q^2 times the continuous mixture density
    (the cell-mass correction is (q/s)^2 / 24 < 1e-10 here), so it equals
    the separately pinned orc_gmm_logpdf plus 2 ln q."""
    for seed in range(5):
        out = inputs.mlp_outputs(seed)
        rng = np.random.default_rng(seed)
        for _ in range(50):
            Dx, Dy = rng.integers(-400000, 400000, 2)
            ref = orc.gmm_logpdf(out, Dx * Q, Dy * Q) + 2 * math.log(Q)
            assert abs(orc.learned_logp(out, Dx, Dy, 26, 0.0) - ref) < 1e-9


def test_logp_branch_weight_is_exact():
    """The branch probability is E / 2^32 with E the nearest integer to
    eps 2^32: on a step-lattice point far from every Gaussian component the
    law is E 2^-32 2^-28 (plus a negligible Gaussian tail)."""
    out = _one_component(0.5, 0.5, -9.0, -9.0)
    m = 26
    for eps in (0.1, 0.25, 1.0 / 3.0, 0.9):
        E = round(float(np.float32(eps)) * 2 ** 32)
        got = orc.learned_logp(out, -m * 101, -m * 55, m, eps)
        assert got == pytest.approx(math.log(E / 2 ** 32) - 28 * LN2, abs=1e-12)


# --------------------------------------------------------------------------
# The draws against the law
def test_draws_follow_lattice_law_narrow_component():
    """A component of width 300 q: the counts of 4e6 draws on every lattice
    cell within 28 q of the mean agree with n P(D) (chi-square), so the draw
    resolves the lattice where the law varies from cell to cell."""
    s = 300 * Q
    out = _one_component(0.01 + 0.3 * Q, -0.02 + 0.6 * Q, math.log(s), math.log(s))
    out = out.astype(np.float32).astype(np.float64)
    n = 4_000_000
    D, drawn, lp = orc.learned_proposals(out, 26, 0.0, 7, n)
    assert drawn.all()
    c = np.rint(out[1:3] / Q).astype(np.int64)
    R = 28
    inwin = (np.abs(D[:, 0] - c[0]) <= R) & (np.abs(D[:, 1] - c[1]) <= R)
    idx = (D[inwin, 0] - c[0] + R) * (2 * R + 1) + (D[inwin, 1] - c[1] + R)
    counts = np.bincount(idx, minlength=(2 * R + 1) ** 2)
    expect = np.array([n * math.exp(orc.learned_logp(out, c[0] + i - R, c[1] + j - R, 26, 0.0))
                       for i in range(2 * R + 1) for j in range(2 * R + 1)])
    assert expect.min() > 5
    x2 = ((counts - expect) ** 2 / expect).sum()
    dof = len(counts)
    assert chi2.sf(x2, dof) > 1e-4, (x2, dof)
    # the logp reported with each draw is the law at the drawn point
    for k in range(0, 1000, 97):
        assert lp[k] == orc.learned_logp(out, D[k, 0], D[k, 1], 26, 0.0)


def _radius_phase(D, nbins=16):
    """Histogram of (Dx^2 + Dy^2) mod 2^21 in nbins equal bins."""
    r2 = D[:, 0] ** 2 + D[:, 1] ** 2
    return np.bincount(((r2 % 2 ** 21) * nbins) >> 21, minlength=nbins)


def _bm24(n, seed, s):
    """Box-Muller on 24-bit single-precision uniforms (a draw that cannot
    resolve the lattice near the mean), rounded to the lattice."""
    rng = np.random.default_rng(seed)
    u1 = ((rng.integers(0, 2 ** 24, n) + 1) / 2.0 ** 24).astype(np.float32)
    u2 = (rng.integers(0, 2 ** 24, n) / 2.0 ** 24).astype(np.float32)
    r = np.sqrt(np.float32(-2) * np.log(u1)).astype(np.float32)
    th = (np.float32(2 * math.pi) * u2).astype(np.float32)
    dx = (np.float32(s) * r * np.cos(th)).astype(np.float32)
    dy = (np.float32(s) * r * np.sin(th)).astype(np.float32)
    return np.stack([np.rint(dx.astype(np.float64) / Q), np.rint(dy.astype(np.float64) / Q)],
                    1).astype(np.int64)


def test_draws_resolve_the_lattice_near_a_wide_mean():
    """A component of width 1 sigma centred on a lattice point: near the mean
    the law is flat over the lattice, so Dx^2 + Dy^2 modulo 2^21 q^2 is
    uniform among draws within 0.02 sigma.  A 24-bit draw puts its radii on
    rings r^2 = k 2^21 q^2 there and fails the same test."""
    out = _one_component(0.0, 0.0, 0.0, 0.0)
    n = 8_000_000
    D, drawn, _ = orc.learned_proposals(out, 26, 0.0, 11, n)
    R2 = (0.02 / Q) ** 2
    near = D[drawn][(D[drawn] ** 2).sum(1) < R2]
    assert len(near) > 1000
    h = _radius_phase(near)
    e = len(near) / len(h)
    assert chi2.sf(((h - e) ** 2 / e).sum(), len(h) - 1) > 1e-4, h
    # the same statistic on a 24-bit Box-Muller draw
    bad = _bm24(n, 12, 1.0)
    near_bad = bad[(bad ** 2).sum(1) < R2]
    hb = _radius_phase(near_bad)
    eb = len(near_bad) / len(hb)
    assert chi2.sf(((hb - eb) ** 2 / eb).sum(), len(hb) - 1) < 1e-12, hb


def test_uniform_branch_draws_are_the_plain_step():
    """eps = 1: every draw is m j per axis with j odd, |j| <= 2^14 - 1, and the
    2^14 values are equally likely."""
    m = 7
    n = 1_000_000
    D, drawn, lp = orc.learned_proposals(inputs.mlp_outputs(2), m, 1.0, 3, n)
    assert drawn.all()
    assert (D % m == 0).all()
    j = D // m
    assert (j % 2 == 1).all() and (np.abs(j) <= 16383).all()
    counts = np.bincount(((j[:, 0] + 16383) // 2), minlength=16384)
    e = n / 16384
    assert chi2.sf(((counts - e) ** 2 / e).sum(), 16383) > 1e-4
    assert np.allclose(lp, -28 * LN2)


def test_mixture_weights_and_failed_draws():
    """Four components far apart: the share of draws near each mean is its
    softmax weight (4 binomial SE); a component centred beyond 1 sigma
    fails about half its draws on that axis."""
    out = np.zeros(20)
    logits = np.array([0.3, -0.7, 1.1, -0.2])
    means = [(-0.5, -0.5), (0.5, -0.5), (-0.5, 0.5), (1.0, 0.5)]
    for k in range(4):
        out[5 * k] = logits[k]
        out[5 * k + 1], out[5 * k + 2] = means[k]
        out[5 * k + 3] = out[5 * k + 4] = -6.0
    pi = np.exp(logits - logits.max())
    pi /= pi.sum()
    n = 400_000
    D, drawn, _ = orc.learned_proposals(out, 26, 0.0, 5, n)
    for k in range(3):
        near = drawn & (np.abs(D[:, 0] * Q - means[k][0]) < 0.05) & \
            (np.abs(D[:, 1] * Q - means[k][1]) < 0.05)
        f = near.mean()
        assert abs(f - pi[k]) < 4 * math.sqrt(pi[k] * (1 - pi[k]) / n), (k, f, pi[k])
    fail = (~drawn).mean()
    assert abs(fail - pi[3] / 2) < 4 * math.sqrt(pi[3] / 2 * (1 - pi[3] / 2) / n), (fail, pi[3])


# --------------------------------------------------------------------------
# The learned sweep
def test_learned_sweep_with_eps_one_is_the_plain_sweep():
    """With the uniform branch always taken the proposal is the plain step
    and the Metropolis-Hastings ratio is 1, so any network gives the plain
    trajectory bit for bit."""
    cfg = dict(N=256, eta=0.60, seed=4, cell_min=3.0, lattice=0, step_m=40)
    a, b = OracleBox(**cfg), OracleBox(**cfg)
    a.sweep(15)
    b.sweep_learned(inputs.mlp_params(8), 1.0, 15)
    for u, v in zip(a.cells(), b.cells()):
        assert np.array_equal(u, v)
    assert a.info()["accepts"] == b.info()["accepts"] > 0


def test_learned_sweep_keeps_two_disks_uniform():
    """N = 2 with an arbitrary network: the Metropolis-Hastings correction
    keeps the separation uniform on the box minus the exclusion disk, so
    P* = (4 eta / pi)(1 - eta)/(1 - 2 eta) (closed form)."""
    b = OracleBox(2, 0.04, seed=9, cell_min=3.0, lattice=2, step_m=200)
    X = np.array([int(1.0 / Q), int(7.5 / Q)], np.int64)
    Y = np.array([int(1.5 / Q), int(8.0 / Q)], np.int64)
    b.set_positions_q(X, Y)
    i = b.info()
    L, eta = i["L_eff"], i["eta_eff"]
    p = inputs.mlp_params(31, scale=0.3)
    K, dr, blocks, nrec = 100, 0.01, 20, 30000
    bc = np.zeros((blocks, K), np.int64)
    for t in range(nrec):
        b.sweep_learned(p, 0.2, 2)
        b.pair_hist(K, dr, bc[t * blocks // nrec])
    assert b.info()["accepts"] > 0.05 * b.info()["trials"]
    per_block = [orc.pressure_fit(c, dr, nrec // blocks, 2, L)["P_star"] for c in bc]
    P, se = mean_se(per_block)
    exact = 4 * eta / math.pi * (1 - eta) / (1 - 2 * eta)
    assert abs(P - exact) < 3 * se, (P, exact, se)
    assert b.count_overlaps() == 0


def test_collecting_sweep_records_accepted_plain_moves():
    """The recording sweep follows the plain trajectory bit for bit; it
    records one move per accepted trial, each a plain step (odd multiples of
    m q) with the features of a valid neighbourhood (at most 12 neighbours
    within 3 sigma, sorted by distance, none closer than contact)."""
    cfg = dict(N=1024, eta=0.65, seed=6, cell_min=3.0, lattice=1, step_m=40)
    a, b = OracleBox(**cfg), OracleBox(**cfg)
    a.sweep(5)
    F, D, tot = b.sweep_collect(5, 100000)
    for u, v in zip(a.cells(), b.cells()):
        assert np.array_equal(u, v)
    assert tot == a.info()["accepts"] == len(F)
    j = np.rint(D.astype(np.float64) / (40 * Q)).astype(np.int64)
    assert np.array_equal(j * 40 * Q, D.astype(np.float64))
    assert (j % 2 == 1).all() and (np.abs(j) < 16384).all()
    r2 = F[:, 0::2].astype(np.float64) ** 2 + F[:, 1::2].astype(np.float64) ** 2
    nz = r2 > 0
    assert (r2[nz] >= 4.0 - 1e-5).all() and (r2 < 9.0).all()
    assert (nz[:, :-1] >= nz[:, 1:]).all()  # padding only at the end
    both = nz[:, 1:]
    assert (r2[:, 1:][both] >= r2[:, :-1][both]).all()  # sorted by distance


# --------------------------------------------------------------------------
# Overlap count, psi field, Adam
def test_count_overlaps_known_pairs():
    """Hand-placed pairs: at 1.9 sigma (overlap), across the periodic edge
    at 1.5 sigma (overlap), at 2 - q (fp32 r^2 < 4: overlap), at exactly
    fp32 r^2 = 4 (contact: allowed), and one triple with two overlaps."""
    b = OracleBox(16, 0.008, lattice=2)
    Lq = b.info()["W"] * b.info()["M"]
    two = 2 * 2 ** 22
    pts = [
        (10 * 2 ** 22, 10 * 2 ** 22), (10 * 2 ** 22 + int(1.9 * 2 ** 22), 10 * 2 ** 22),  # 1.9
        (2 ** 21, 20 * 2 ** 22), (Lq - 2 ** 20, 20 * 2 ** 22 + 3 * 2 ** 20),             # edge
        (30 * 2 ** 22, 5 * 2 ** 22), (30 * 2 ** 22 + two - 1, 5 * 2 ** 22),             # 2 - q
        (5 * 2 ** 22, 30 * 2 ** 22), (5 * 2 ** 22, 30 * 2 ** 22 + two),                 # contact
        (20 * 2 ** 22, 30 * 2 ** 22), (20 * 2 ** 22 + 2 ** 22, 30 * 2 ** 22),           # triple
        (20 * 2 ** 22 + 2 ** 23 + 2 ** 21, 30 * 2 ** 22),
    ]
    n = 16
    X = np.array([p[0] for p in pts] + [(40 + 5 * k) * 2 ** 22 for k in range(n - len(pts))],
                 np.int64)
    Y = np.array([p[1] for p in pts] + [40 * 2 ** 22 for k in range(n - len(pts))], np.int64)
    assert Lq > 70 * 2 ** 22
    b.set_positions_q(X, Y)
    assert b.count_overlaps() == 5
    # the contact pair alone: none
    c = OracleBox(16, 0.008, lattice=2)
    X2, Y2 = X.copy(), Y.copy()
    for k in range(len(pts)):
        if k not in (6, 7):
            X2[k], Y2[k] = (10 + 5 * k) * 2 ** 22, 60 * 2 ** 22
    c.set_positions_q(X2, Y2)
    assert c.count_overlaps() == 0


def test_psi6_field_impulse_and_constant():
    """One disk per cell (N = M^2): a psi of 1 on one disk and 0 elsewhere
    gives 1/9 on exactly the 3 x 3 cells around its cell; a constant psi
    gives the constant in every cell."""
    b = OracleBox(256, 0.70, lattice=0)
    i = b.info()
    M = i["M"]
    assert M == 16 and (b.cells()[0] == 1).all()
    cnt, tag, _, _ = b.cells()
    for t in (0, 17, 255):
        c = int(np.where(tag[:, 0] == t)[0][0])
        psi = np.zeros(256, complex)
        psi[t] = 1.0
        f = b.psi6_field(psi)
        ci, cj = c % M, c // M
        expect = np.zeros(M * M)
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                expect[(ci + di) % M + M * ((cj + dj) % M)] = 1.0 / 9.0
        assert np.allclose(f, expect, atol=1e-15)
    f = b.psi6_field(np.full(256, 0.3 - 0.4j))
    assert np.allclose(f, 0.3 - 0.4j, atol=1e-15)


def test_psi6_and_field_of_the_stretched_triangular_start():
    """The triangular start stretched to the square box has every disk's six
    nearest neighbours at (+-h, 0) and (+-h/2, +-h): psi_j =
    (2 + 4 cos 6 atan 2) / 6 = 718/750 for every disk, and so in every cell
    of the field (floor placement moves disks by < q: 1e-6 tolerance)."""
    b = OracleBox(1024, 0.5, lattice=1)
    psi = b.psi6()
    assert np.abs(psi - 718.0 / 750.0).max() < 1e-6
    f = b.psi6_field(psi)
    cnt = b.cells()[0]
    M = b.info()["M"]
    occupied_block = np.zeros(M * M, bool)
    for c in np.nonzero(cnt)[0]:
        ci, cj = c % M, c // M
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                occupied_block[(ci + di) % M + M * ((cj + dj) % M)] = True
    assert np.abs(f[occupied_block] - 718.0 / 750.0).max() < 1e-6
    assert (f[~occupied_block] == 0).all()


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments stay g and g^2 at
    every step t, so after t steps each parameter has moved by
    t lr g / (|g| + 1e-8)."""
    p = np.linspace(-1, 1, 40)
    g = np.linspace(-2, 3, 40)
    m, v = np.zeros(40), np.zeros(40)
    p0 = p.copy()
    for t in range(1, 26):
        orc.adam(p, m, v, g, 1e-3, t)
        assert np.allclose(p, p0 - t * 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13), t
