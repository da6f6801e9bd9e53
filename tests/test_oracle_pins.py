"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known answers, an independent Philox implementation, closed forms (N = 2,
lattices, exact polynomials, AR(1)), brute force on tiny inputs, an exact
direct sampler, and the low-density virial series of hard disks.
"""
import ctypes as C
import math
import os

import numpy as np
import pytest

from oracle import orc
from oracle.orc import OracleBox, Q
from tests.stats import block_mean_se, mean_se

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Philox4x32-10
def test_philox_known_answers():
    path = os.path.join(HERE, "golden", "philox_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        key = v[0] | (v[1] << 32)
        out = orc.philox(key, v[2:6])
        assert [int(o) for o in out] == v[6:10]


def test_philox_matches_rocrand_engine():
    from tests.pins.build import build
    ref = C.CDLL(build())
    rng = np.random.default_rng(12345)
    for _ in range(3000):
        key = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        ctr = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64).astype(np.uint32)
        out = np.zeros(4, np.uint32)
        ref.ref_philox(C.c_uint32(key & 0xFFFFFFFF), C.c_uint32(key >> 32),
                       ctr.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p))
        assert (orc.philox(key, ctr) == out).all()


# --------------------------------------------------------------------------
# Geometry (Sec. II.A: eta = N pi sigma^2 / L^2; Sec. II.B: w >~ 2 sigma)
@pytest.mark.parametrize("N,eta,M_expected", [
    (256, 0.60, 18), (65536, 0.716, 268), (1048576, 0.716, 1072), (1048576, 0.700, 1084),
    (1048576, 0.720, 1068), (4096, 0.69, 68)])
def test_geometry_closed_form(N, eta, M_expected):
    g = orc.geometry(N, eta)
    L = math.sqrt(N * math.pi / eta)
    assert abs(g["L"] - L) < 1e-9 * L
    assert g["M"] == M_expected and g["M"] % 2 == 0
    # largest even M with L / M >= 2
    assert L / g["M"] >= 2.0 and L / (g["M"] + 2) < 2.0
    # w on the q lattice, nearest to L / M, and exactly representable in fp32
    assert abs(g["W"] * Q - L / g["M"]) <= Q / 2 + 1e-15
    assert float(np.float32(g["w"])) == g["w"]
    assert g["cap"] == 4  # w < 2 sqrt 2: at most four disks per cell


def test_geometry_rejects():
    with pytest.raises(ValueError):
        orc.geometry(0, 0.5)
    with pytest.raises(ValueError):
        orc.geometry(16, 0.79)          # above pi/4
    with pytest.raises(ValueError):
        orc.geometry(4, 0.5)            # M < 4
    with pytest.raises(ValueError):
        OracleBox(255, 0.5, lattice=0)  # lattice start needs a square N


def test_learned_grid_capacity():
    g = orc.geometry(65536, 0.716, cell_min=3.0)
    assert g["M"] == 178 and 3.0 <= g["w"] < 3.02
    assert g["cap"] == 5  # 2 sqrt 2 <= w < 3.328: five disks fit, six do not


# --------------------------------------------------------------------------
# Lattice start and sweep invariants
def _min_image(d, Lq):
    d = np.mod(d, Lq)
    return np.where(2 * d > Lq, d - Lq, d)


@pytest.mark.parametrize("N,eta,lattice", [(256, 0.6, 0), (1024, 0.716, 1), (4096, 0.78, 1)])
def test_lattice_start_valid(N, eta, lattice):
    b = OracleBox(N, eta, lattice=lattice)
    assert b.count_overlaps() == 0
    cnt, tag, x, y = b.cells()
    i = b.info()
    assert cnt.sum() == N
    tags = np.concatenate([tag[c, :cnt[c]] for c in range(len(cnt))])
    assert sorted(tags.tolist()) == list(range(N))
    for c in range(len(cnt)):
        assert (np.diff(tag[c, :cnt[c]].astype(np.int64)) > 0).all()  # tag order at start
    assert (x >= 0).all() and (x < i["w"]).all() and (y >= 0).all() and (y < i["w"]).all()
    # the nearest-neighbour spacing of the start is L / sqrt(N)
    X, Y = b.positions_q()
    n = int(round(math.sqrt(N)))
    dX = _min_image(X[1] - X[0], i["W"] * i["M"])
    assert abs(dX * Q - i["L_eff"] / n) <= 2 * Q


def test_sweep_moves_each_disk_at_most_one_step():
    """With one trial per cell, a disk moves at most once per sweep, by less
    than d per axis; the grid shift changes no absolute position."""
    b = OracleBox(1024, 0.70, seed=3, lattice=1, step_m=26)
    Lq = b.info()["W"] * b.info()["M"]
    D = 26 * 2 ** 14  # d in q units
    X0, Y0 = b.positions_q()
    for _ in range(20):
        b.sweep(1)
        X1, Y1 = b.positions_q()
        dx, dy = _min_image(X1 - X0, Lq), _min_image(Y1 - Y0, Lq)
        assert np.abs(dx).max() < D and np.abs(dy).max() < D
        moved = (dx != 0) | (dy != 0)
        assert moved.sum() > 0
        X0, Y0 = X1, Y1
    cnt, tag, x, y = b.cells()
    assert cnt.sum() == 1024 and cnt.max() <= 4
    w = b.info()["w"]
    for c in np.nonzero(cnt)[0]:
        assert (x[c, :cnt[c]] < w).all() and (x[c, :cnt[c]] >= 0).all()
    assert b.count_overlaps() == 0


@pytest.mark.parametrize("n_trial", [1, 3])
def test_same_colour_cells_are_independent(n_trial):
    """The result of a sweep does not depend on the order in which the cells of
    one colour are visited (Sec. II.B: same-colour cells are >= w apart)."""
    boxes = [OracleBox(1024, 0.71, seed=7, lattice=1, step_m=40, n_trial=n_trial)
             for _ in range(3)]
    for order, b in enumerate(boxes):
        b.sweep(30, cell_order=order)
    ref = boxes[0].cells()
    for b in boxes[1:]:
        for a, c in zip(ref, b.cells()):
            assert np.array_equal(a, c)
    assert boxes[0].info()["accepts"] > 0


def test_dense_sweeps_keep_no_overlaps():
    b = OracleBox(4096, 0.716, seed=1, lattice=1, step_m=20)
    b.sweep(50)
    assert b.count_overlaps() == 0
    i = b.info()
    assert 0.2 < i["accepts"] / i["trials"] < 0.8


# --------------------------------------------------------------------------
# Histogram counting (Eq. (2)) on a lattice with known distances
def test_pair_hist_square_lattice():
    b = OracleBox(256, 0.60, lattice=0)
    i = b.info()
    h = i["L_eff"] / 16
    K, dr = 150, 0.01  # r in [2, 3.5)
    counts = b.pair_hist(K, dr)
    r = 2 + (np.arange(K) + 0.5) * dr
    near = np.abs(r - h) < 0.02
    diag = np.abs(r - h * math.sqrt(2)) < 0.02
    # every disk has 4 axis neighbours at h and 4 diagonal ones at h sqrt 2;
    # unordered pairs: 2N of each
    assert counts[near].sum() == 2 * 256
    assert counts[diag].sum() == 2 * 256
    assert counts.sum() == 4 * 256
    # ordered counts from a subset: every disk contributes 8
    sel = np.zeros(256, np.uint8)
    sel[::7] = 1
    sub = b.pair_hist_subset(sel, K, dr)
    assert sub.sum() == 8 * sel.sum()


def test_hist_edges():
    E = orc.hist_edges(100, 1e-3)
    assert E[0] == np.float32(4.0)
    assert np.allclose(E.astype(np.float64), (2 + np.arange(101) * 1e-3) ** 2, rtol=1e-7)


# --------------------------------------------------------------------------
# Contact fit (Sec. II.C.1): exact polynomials are recovered
def _counts_from_g(gfun, K, dr, N, L, n_conf):
    r = 2 + (np.arange(K) + 0.5) * dr
    p = 0.5 * N * (N - 1) * n_conf
    return np.rint(gfun(r) * p * 2 * np.pi * r * dr / L ** 2).astype(np.int64)


def test_fit_recovers_quartic():
    N, L, n_conf, K, dr = 1000, 60.0, 10 ** 12, 100, 1e-3
    coef = [6.6755, -31.0, 120.0, -400.0, 900.0]
    g = lambda r: sum(c * (r - 2) ** e for e, c in enumerate(coef))
    res = orc.pressure_fit(_counts_from_g(g, K, dr, N, L, n_conf), dr, n_conf, N, L)
    assert abs(res["g_contact"] - coef[0]) < 1e-9
    assert np.allclose(res["coef"], coef, rtol=1e-5, atol=1e-6)
    eta = N * math.pi / L ** 2
    Z = 1 + 2 * eta * (N - 1) / N * coef[0]
    assert abs(res["Z"] - Z) < 1e-9 and abs(res["P_star"] - 4 * eta * Z / math.pi) < 1e-9


def test_fit_flat_gives_n2_pressure():
    """For N = 2 the separation is uniform outside the excluded disk, so
    g = 1 / (1 - 2 eta) exactly and Z = (1 - eta) / (1 - 2 eta)."""
    N, L = 2, 11.21
    eta = 2 * math.pi / L ** 2
    n_conf = 10 ** 15
    res = orc.pressure_fit(_counts_from_g(lambda r: 0 * r + 1 / (1 - 2 * eta), 100, 0.01, N, L,
                                          n_conf), 0.01, n_conf, N, L)
    assert abs(res["Z"] - (1 - eta) / (1 - 2 * eta)) < 1e-9


# --------------------------------------------------------------------------
# psi_6 (Eq. (8)) on a triangular patch, and under rotation
def _triangular_patch(n, a, theta, centre):
    pts = []
    for r in range(n):
        for c in range(n):
            u = (c + 0.5 * (r % 2)) * a - n * a / 2
            v = r * a * math.sqrt(3) / 2 - n * a * math.sqrt(3) / 4
            pts.append((u, v))
    pts = np.array(pts)
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    return pts @ R.T + centre


@pytest.mark.parametrize("theta", [0.0, 0.2, 1.1])
def test_psi6_triangular_patch(theta):
    n = 9
    N = n * n
    b = OracleBox(N, 0.05, lattice=2)
    L = b.info()["L_eff"]
    P = _triangular_patch(n, 2.3, theta, np.array([L / 2, L / 2]))
    b.set_positions_q(np.rint(P[:, 0] / Q).astype(np.int64), np.rint(P[:, 1] / Q).astype(np.int64))
    psi = b.psi6()
    interior = [r * n + c for r in range(2, n - 2) for c in range(2, n - 2)]
    expect = np.exp(6j * theta)
    assert np.abs(psi[interior] - expect).max() < 1e-5
    # a disk with only three lattice neighbours on one side is not 6-fold
    assert abs(psi[0]) < 0.9


def test_psi6_rotation_covariance():
    b = OracleBox(64, 0.3, seed=2, lattice=0, step_m=60)
    b.sweep(40)
    X, Y = b.positions_q()
    L = b.info()["L_eff"]
    psi0 = b.psi6()
    # rotate by 90 degrees about the box centre: a symmetry of the periodic
    # square box; exp(6 i phi) picks up exp(6 i pi/2) = -1
    Lq = b.info()["W"] * b.info()["M"]
    b.set_positions_q((Lq - Y) % Lq, X.copy())
    psi1 = b.psi6()
    assert np.abs(psi1 + psi0).max() < 1e-9
    assert np.abs(psi0).mean() > 0.05 and L > 0


# --------------------------------------------------------------------------
# C(dt) (Eq. (9)) and tau on an AR(1) series with tau = -1 / ln(phi)
def test_acf_tau_ar1():
    rng = np.random.default_rng(0)
    phi, n = 0.95, 400000
    e = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    s = np.empty(n, np.complex128)
    s[0] = e[0]
    for t in range(1, n):
        s[t] = phi * s[t - 1] + e[t]
    Cv = orc.acf(s, 200)
    assert abs(Cv[0] - 1) < 1e-12
    assert np.allclose(Cv[:60], phi ** np.arange(60), atol=0.02)
    tau = orc.tau_fit(Cv, 0.05, 0.5)
    assert abs(tau - (-1 / math.log(phi))) / (-1 / math.log(phi)) < 0.05
    ti = orc.tau_int(Cv, 6.0)
    assert abs(ti - (1 + phi) / (2 * (1 - phi))) / ((1 + phi) / (2 * (1 - phi))) < 0.1


# --------------------------------------------------------------------------
# Statistical pins of the sampler.
def _n2_box(eta, seed):
    b = OracleBox(2, eta, seed=seed, lattice=2, step_m=255)
    i = b.info()
    X = np.array([int(1.0 / Q), int(5.5 / Q)], np.int64)
    Y = np.array([int(1.0 / Q), int(6.0 / Q)], np.int64)
    b.set_positions_q(X, Y)
    return b, i


def test_n2_uniform_separation_and_pressure():
    """N = 2: the separation vector is uniform on the box minus the disk of
    radius 2, so g is flat at 1/(1 - 2 eta) and P* = (4 eta/pi)(1-eta)/(1-2eta)."""
    b, i = _n2_box(0.05, seed=11)
    L, Lq, eta = i["L_eff"], i["W"] * i["M"], i["eta_eff"]
    K, dr = 100, 0.01
    nrec, thin = 200000, 3
    seps = np.empty((nrec, 2))
    blocks = 20
    bcounts = np.zeros((blocks, K), np.int64)
    for t in range(nrec):
        b.sweep(thin)
        X, Y = b.positions_q()
        seps[t] = _min_image(X[1] - X[0], Lq) * Q, _min_image(Y[1] - Y[0], Lq) * Q
        b.pair_hist(K, dr, bcounts[t * blocks // nrec])
    r = np.hypot(seps[:, 0], seps[:, 1])
    assert r.min() >= 2.0
    # radial: fraction with r < 3 against the area ratio
    frac, se = block_mean_se((r < 3.0).astype(float))
    expect = math.pi * (9 - 4) / (L * L - 4 * math.pi)
    assert abs(frac - expect) < 3 * se, (frac, expect, se)
    # quadrants of the separation vector are equally likely
    for q_ in [(seps[:, 0] > 0) & (seps[:, 1] > 0), (seps[:, 0] < 0) & (seps[:, 1] > 0)]:
        m, s = block_mean_se(q_.astype(float))
        assert abs(m - 0.25) < 3 * s
    # pressure through the whole contact-fit pipeline, SE from block estimates
    per_block = [orc.pressure_fit(bc, dr, nrec // blocks, 2, L)["P_star"] for bc in bcounts]
    P, se = mean_se(per_block)
    P_exact = 4 * eta / math.pi * (1 - eta) / (1 - 2 * eta)
    assert abs(P - P_exact) < 3 * se, (P, P_exact, se)


def _direct_samples(N, L, nsamp, rng):
    out = []
    while sum(len(o) for o in out) < nsamp:
        P = rng.uniform(0, L, size=(200000, N, 2))
        d = P[:, :, None, :] - P[:, None, :, :]
        d -= L * np.rint(d / L)
        r2 = (d ** 2).sum(-1)
        iu = np.triu_indices(N, 1)
        ok = (r2[:, iu[0], iu[1]] >= 4.0).all(axis=1)
        out.append(P[ok])
    return np.concatenate(out)[:nsamp]


def test_matches_direct_sampling_small_n():
    """For N = 9 at eta = 0.15, placing all disks at random and rejecting any
    overlapping configuration samples the same uniform measure exactly."""
    N, eta = 9, 0.15
    b = OracleBox(N, eta, seed=21, lattice=0, step_m=128)
    i = b.info()
    L, Lq = i["L_eff"], i["W"] * i["M"]
    edges = np.array([2.0, 2.25, 2.5, 3.0, 3.5, 4.5, 6.0])
    iu = np.triu_indices(N, 1)

    def binned(X, Y):
        dx = _min_image(X[:, None] - X[None, :], Lq) * Q
        dy = _min_image(Y[:, None] - Y[None, :], Lq) * Q
        r = np.hypot(dx, dy)[iu]
        return np.histogram(r, edges)[0]

    b.sweep(200)
    mc = []
    for _ in range(60000):
        b.sweep(2)
        mc.append(binned(*b.positions_q()))
    mc = np.array(mc, float)
    ds = _direct_samples(N, L, 60000, np.random.default_rng(5))
    dsb = []
    for P in ds:
        X = np.rint(P[:, 0] / Q).astype(np.int64)
        Y = np.rint(P[:, 1] / Q).astype(np.int64)
        dsb.append(binned(X, Y))
    dsb = np.array(dsb, float)
    for k in range(len(edges) - 1):
        m1, s1 = block_mean_se(mc[:, k])
        m2, s2 = mean_se(dsb[:, k])
        assert abs(m1 - m2) < 3 * math.hypot(s1, s2), (k, m1, m2, s1, s2)


def test_virial_series_low_density():
    """Z = 1 + 2 eta + 3.128 eta^2 + 4.258 eta^3 + R with the positive
    remainder R of the next terms (5.337, 6.363, 7.351, 8.31 times
    eta^4..eta^7) for hard disks at eta <= 0.2."""
    eta, N = 0.2, 1024
    b = OracleBox(N, eta, seed=9, lattice=0, step_m=128)
    i = b.info()
    e = i["eta_eff"]
    K, dr = 20, 0.01
    b.sweep(300)
    nconf, blocks = 12000, 12
    bc = np.zeros((blocks, K), np.int64)
    for t in range(nconf):
        b.sweep(2)
        b.pair_hist(K, dr, bc[t * blocks // nconf])
    Zs = [orc.pressure_fit(c, dr, nconf // blocks, N, i["L_eff"])["Z"] for c in bc]
    Z, se = mean_se(Zs)
    series = 1 + 2 * e + 3.128 * e ** 2 + 4.258 * e ** 3
    rem = 5.337 * e ** 4 + 6.363 * e ** 5 + 7.351 * e ** 6 + 8.31 * e ** 7
    assert -3 * se <= Z - series <= 3 * se + 1.1 * rem, (Z, series, rem, se)
    assert se < 0.01


# --------------------------------------------------------------------------
# Learned proposal reference: features, MLP, mixture density, gradients, Adam
def test_features_bruteforce_tiny():
    b = OracleBox(4, 0.02, lattice=2, cell_min=3.0)
    W, M = b.info()["W"], b.info()["M"]
    w = W * Q
    # disk 0 in cell (1, 1) at local (1.5, 1.5); neighbours at known offsets
    base = np.array([w + 1.5, w + 1.5])
    offs = np.array([[0.0, 0.0], [2.5, 0.0], [0.0, -2.1], [-1.8, 1.9]])
    P = base + offs
    b.set_positions_q(np.rint(P[:, 0] / Q).astype(np.int64), np.rint(P[:, 1] / Q).astype(np.int64))
    f, n = b.features(1 + M * 1, 0, np.float32(1.5), np.float32(1.5))
    assert n == 3
    order = np.argsort(np.hypot(offs[1:, 0], offs[1:, 1]))
    exp = offs[1:][order].ravel()
    assert np.allclose(f[:6], exp, atol=1e-6) and (f[6:] == 0).all()
    # a trial position moves every feature by the opposite displacement
    f2, n2 = b.features(1 + M, 0, np.float32(1.75), np.float32(1.25))
    assert n2 == 3 and np.allclose(f2[:6], exp - np.tile([0.25, -0.25], 3), atol=1e-6)


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(orc.NPARAM) * scale


def test_mlp_special_cases():
    p = np.zeros(orc.NPARAM)
    b3 = np.arange(20) * 0.1
    p[-20:] = b3
    assert np.allclose(orc.mlp_forward(p, np.ones(24)), b3)
    # one path: f0 -> unit 0 -> unit 0 -> output 1, SiLU(v) = v / (1 + e^-v)
    p = np.zeros(orc.NPARAM)
    p[0] = 2.0                      # W1[0][0]
    p[64 * 24 + 64] = 1.5           # W2[0][0]
    p[64 * 24 + 64 + 4096 + 64 + 64] = 0.7   # W3[1][0]
    f = np.zeros(24)
    f[0] = 0.8
    silu = lambda v: v / (1 + math.exp(-v))
    out = orc.mlp_forward(p, f)
    assert abs(out[1] - 0.7 * silu(1.5 * silu(1.6))) < 1e-14
    assert np.count_nonzero(out) == 1


def test_gmm_logpdf_reduces_to_gaussian():
    from scipy.stats import multivariate_normal
    out = np.zeros(20)
    out[0:5] = [0.0, 0.03, -0.02, math.log(0.05), math.log(0.08)]
    for k in range(1, 4):
        out[5 * k] = -800.0
    for dx, dy in [(0.0, 0.0), (0.1, -0.05), (-0.07, 0.2)]:
        ref = multivariate_normal([0.03, -0.02], np.diag([0.05 ** 2, 0.08 ** 2])).logpdf([dx, dy])
        assert abs(orc.gmm_logpdf(out, dx, dy) - ref) < 1e-10
    # four identical components equal one
    for k in range(1, 4):
        out[5 * k:5 * k + 5] = out[0:5]
    ref = multivariate_normal([0.03, -0.02], np.diag([0.05 ** 2, 0.08 ** 2])).logpdf([0.01, 0.02])
    assert abs(orc.gmm_logpdf(out, 0.01, 0.02) - ref) < 1e-10


def test_nll_gradient_finite_differences():
    rng = np.random.default_rng(8)
    p = _params(3, 0.2)
    F = rng.uniform(-2.5, 2.5, size=(6, 24))
    D = rng.normal(0, 0.1, size=(6, 2))
    loss, g = orc.nll_grad(p, F, D)
    # check the loss itself against the mixture density
    ref = -np.mean([orc.gmm_logpdf(orc.mlp_forward(p, F[b]), *D[b]) for b in range(6)])
    assert abs(loss - ref) < 1e-12
    idx = np.concatenate([rng.choice(orc.NPARAM, 60, replace=False), np.arange(orc.NPARAM - 20, orc.NPARAM)])
    h = 1e-6
    for e in idx:
        pp, pm = p.copy(), p.copy()
        pp[e] += h
        pm[e] -= h
        fd = (orc.nll_grad(pp, F, D)[0] - orc.nll_grad(pm, F, D)[0]) / (2 * h)
        assert abs(fd - g[e]) <= 1e-6 * max(1.0, abs(fd)), (e, fd, g[e])


def test_adam_first_step():
    """At t = 1 the bias-corrected moments are g and g^2, so every parameter
    moves by lr * g / (|g| + eps)."""
    p = np.linspace(-1, 1, 50)
    g = np.linspace(-3, 2, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    p0 = p.copy()
    orc.adam(p, m, v, g, 1e-3, 1)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-15)


# --------------------------------------------------------------------------
# Positional order: S(q) and chi_j (Sec. IV.C), C_q(r) (Sec. IV.D)
def _square_lattice(n, eta):
    """n x n square lattice placed at (i + 1/2) Lq / n in q units."""
    b = OracleBox(n * n, eta, lattice=2)
    Lq = b.info()["W"] * b.info()["M"]
    i = np.arange(n)
    X = ((2 * i + 1) * Lq) // (2 * n)
    XX, YY = np.meshgrid(X, X)
    b.set_positions_q(XX.ravel(), YY.ravel())
    return b, Lq


def test_structure_factor_square_lattice_selection_rules():
    """On an n x n lattice, rho(q) factorises into two geometric sums that
    vanish unless h and k are both multiples of n; at (n, 0), (0, n) and
    (n, n) every phase agrees (S = N up to the sub-q placement)."""
    n = 16
    b, Lq = _square_lattice(n, 0.5)
    hk = [(n, 0), (0, n), (n, n), (2 * n, -n), (1, 0), (0, 3), (5, 7), (n + 1, 0), (n, 1)]
    S = b.structure_factor(hk)
    N = n * n
    for (h, k), s in zip(hk, S):
        if h % n == 0 and k % n == 0:
            assert abs(s - N) < 1e-6 * N, (h, k, s)
        else:
            assert s < 1e-6 * N, (h, k, s)


def test_structure_factor_two_disks_closed_form():
    """N = 2: S(q) = |e^{i phi_1} + e^{i phi_2}|^2 / 2 = 1 + cos(q.(x_1 - x_2))."""
    b = OracleBox(2, 0.04, lattice=2)
    i = b.info()
    Lq = i["W"] * i["M"]
    X = np.array([123456789, 987654321], np.int64) % Lq
    Y = np.array([55555555, 33333333], np.int64) % Lq
    b.set_positions_q(X, Y)
    hk = np.array([(1, 0), (3, -2), (7, 11), (-5, 4)], np.int32)
    S = b.structure_factor(hk)
    for (h, k), s in zip(hk, S):
        dph = 2 * math.pi * ((h * (X[0] - X[1]) + k * (Y[0] - Y[1])) % Lq) / Lq
        assert abs(s - (1 + math.cos(dph))) < 1e-12


def test_structure_factor_ideal_gas_mean_one():
    """Uniform independent positions: <S(q)> = 1 for every q != 0."""
    rng = np.random.default_rng(5)
    b = OracleBox(4096, 0.05, lattice=2)
    i = b.info()
    Lq = i["W"] * i["M"]
    X = rng.integers(0, Lq, 4096)
    Y = rng.integers(0, Lq, 4096)
    b.set_positions_q(X, Y)
    hk = [(h, k) for h in range(1, 21) for k in range(-10, 10)]
    S = b.structure_factor(hk)
    # S is exponential with mean 1 for each q: 400 samples
    assert abs(S.mean() - 1.0) < 4 * S.std() / math.sqrt(len(S))


def test_chi_square_lattice():
    n = 16
    b, Lq = _square_lattice(n, 0.5)
    chi = b.chi(n, 0)
    # phases 2 pi (i + 1/2): chi = -1 for every disk
    assert np.abs(chi + 1).max() < 1e-6
    assert np.abs(np.abs(b.chi(3, 5)) - 1).max() < 1e-12


def test_cq_square_lattice_and_pair_counts():
    """On the square lattice with q = (2 pi / a)(1, 0), q.d is a multiple of
    2 pi for every pair, so C_q(r) = 1 wherever pairs exist; the pair counts
    per window agree with a direct count of the lattice distances."""
    n = 16
    b, Lq = _square_lattice(n, 0.5)
    L = Lq * Q
    a = L / n
    dr, B = 0.25, 40
    num, cnt = b.cq(2 * math.pi / a, 0.0, dr, B)
    assert cnt.sum() > 0
    ok = cnt > 0
    assert np.abs(num[ok] / cnt[ok] - 1).max() < 1e-9
    # direct count: lattice displacement vectors (minimum image)
    d = []
    for di in range(-n // 2 + 1, n // 2 + 1):
        for dj in range(-n // 2 + 1, n // 2 + 1):
            if di == 0 and dj == 0:
                continue
            d.append(a * math.hypot(di, dj))
    d = np.array(d)
    ref = np.array([((d >= bb * dr - 1) & (d <= bb * dr + 1)).sum() for bb in range(B)])
    # every disk sees the same displacements: unordered pairs = N * ref / 2
    assert np.array_equal(cnt, n * n * ref // 2)


def test_cq_two_disks():
    b = OracleBox(2, 0.04, lattice=2)
    i = b.info()
    Lq = i["W"] * i["M"]
    X = np.array([2 << 22, (2 << 22) + int(3.3 * (1 << 22))], np.int64)
    Y = np.array([2 << 22, (2 << 22) + int(1.7 * (1 << 22))], np.int64)
    b.set_positions_q(X, Y)
    qx, qy = 1.3, -0.4
    num, cnt = b.cq(qx, qy, 0.5, 10)
    dx, dy = (X[1] - X[0]) * Q, (Y[1] - Y[0]) * Q
    r = math.hypot(dx, dy)
    for bb in range(10):
        inside = bb * 0.5 - 1 <= r <= bb * 0.5 + 1
        assert cnt[bb] == (1 if inside else 0)
        assert abs(num[bb] - (math.cos(qx * dx + qy * dy) if inside else 0.0)) < 1e-12
