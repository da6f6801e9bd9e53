"""Positional order (Sec. IV.C, IV.D) through the C ABI against the oracle, on
states that both sides reach by the same bit-exact trajectory.

Tolerances follow from the arithmetic: the GPU evaluates each term of the
structure factor as an fp32 table root of unity rotated by an fp32 residual
angle from the fp64 phase (absolute error below 1e-6 per term), so |dS| <= 2e-6 sqrt(N S) + 1e-12 N; chi_j is returned in
fp32 (error below 1e-6); C_q sums fp64 cosines in another order
(|d num| <= 1e-12 per pair) and its pair counts are exact.
"""
import math

import numpy as np
import pytest

from oracle.orc import OracleBox

pytestmark = pytest.mark.gpu

SMALL = dict(N=256, eta=0.60, seed=0, lattice=0, step_m=26)
MEDIUM = dict(N=16384, eta=0.716, seed=1, lattice=1, step_m=20)


def boxes(mp, cfg, sweeps):
    g = mp.Box(cfg["N"], cfg["eta"], seed=cfg["seed"], step_m=cfg["step_m"],
               lattice={0: "square", 1: "triangular"}[cfg["lattice"]])
    o = OracleBox(**cfg)
    g.sweep(sweeps)
    o.sweep(sweeps)
    gX, gY = g.positions_q()
    oX, oY = o.positions_q()
    assert np.array_equal(gX, oX) and np.array_equal(gY, oY)
    return g, o


def s_tol(N, S):
    return 2e-6 * np.sqrt(N * np.maximum(S, 0.0)) + 1e-12 * N + 1e-12


@pytest.fixture(scope="module")
def small(gpu_lib):
    return boxes(gpu_lib, SMALL, 200)


@pytest.fixture(scope="module")
def medium(gpu_lib):
    return boxes(gpu_lib, MEDIUM, 20)


def test_structure_factor_small_box(small):
    g, o = small
    N = SMALL["N"]
    h, k = np.meshgrid(np.arange(-12, 13), np.arange(-12, 13))
    hk = np.stack([h.ravel(), k.ravel()], 1)
    hk = np.concatenate([hk, [[4095, -4095], [-4095, 1], [16, 0], [0, 16]]])  # ragged: 629
    S = g.structure_factor(hk)
    So = o.structure_factor(hk)
    assert np.all(np.abs(S - So) <= s_tol(N, So))
    zero = np.nonzero((hk[:, 0] == 0) & (hk[:, 1] == 0))[0][0]
    assert abs(S[zero] - N) <= 1e-9 * N   # every term is exactly 1


def test_structure_factor_chunked_launches(small):
    """More wave vectors than one launch takes (65536): chunk boundaries."""
    g, o = small
    rng = np.random.default_rng(5)
    hk = rng.integers(-4095, 4096, size=(70001, 2)).astype(np.int32)
    S = g.structure_factor(hk)
    So = o.structure_factor(hk)
    assert np.all(np.abs(S - So) <= s_tol(SMALL["N"], So))


def test_structure_factor_rejects_large_index(gpu_lib, small):
    g, _ = small
    with pytest.raises(gpu_lib.MPMCError):
        g.structure_factor([[4096, 0]])
    assert len(g.structure_factor(np.zeros((0, 2), np.int32))) == 0


def test_structure_factor_medium_box(medium):
    g, o = medium
    N = MEDIUM["N"]
    rng = np.random.default_rng(2)
    hk = rng.integers(-300, 301, size=(300, 2))
    S = g.structure_factor(hk)
    So = o.structure_factor(hk)
    assert np.all(np.abs(S - So) <= s_tol(N, So))


def window(L, q_lo, q_hi, theta0, dtheta):
    unit = 2 * math.pi / L
    r = int(math.ceil(q_hi / unit))
    k, h = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
    h, k = h.ravel(), k.ravel()
    n2 = h.astype(np.float64) ** 2 + k.astype(np.float64) ** 2
    keep = (n2 >= (q_lo / unit) ** 2) & (n2 <= (q_hi / unit) ** 2) & (n2 > 0)
    a = np.mod(np.arctan2(k, h) - theta0, 2 * math.pi)
    keep &= a < dtheta
    return np.stack([h[keep], k[keep]], 1)


def test_find_q0_is_the_peak(medium):
    """The first diffraction peak in a 60 degree sector of the annulus
    around 4 pi / (sqrt(3) a0), a0 the triangular lattice constant."""
    g, o = medium
    N = MEDIUM["N"]
    L = o.info()["L_eff"]
    a0 = math.sqrt(2.0 / (math.sqrt(3.0) * N / L ** 2))
    qp = 4 * math.pi / (math.sqrt(3.0) * a0)
    lo, hi, t0, dt = 0.9 * qp, 1.1 * qp, 0.0, math.pi / 3
    h, k, S = g.find_q0(lo, hi, t0, dt)
    cand = window(L, lo, hi, t0, dt)
    So = o.structure_factor(cand)
    assert any((cand[:, 0] == h) & (cand[:, 1] == k))
    mine = o.structure_factor([[h, k]])[0]
    assert abs(S - mine) <= s_tol(N, mine)
    assert mine >= So.max() - 2 * s_tol(N, So.max())
    assert So.max() > 50.0   # a real Bragg peak, far above the liquid's O(1)


def test_chi_and_field(small, medium):
    for g, o in (small, medium):
        for h, k in ((3, -2), (0, 0), (-4095, 4095)):
            chi, field = g.chi_field(h, k)
            ochi = o.chi(h, k)
            assert np.abs(chi - ochi).max() < 1e-6
            assert np.abs(field - o.psi6_field(ochi)).max() < 1e-6


def check_cq(g, o, qx, qy, dr, B):
    num, cnt = g.cq(qx, qy, dr, B)
    onum, ocnt = o.cq(qx, qy, dr, B)
    assert np.array_equal(cnt, ocnt)
    assert np.all(np.abs(num - onum) <= 1e-12 * np.maximum(ocnt, 1))
    return num, cnt


def test_cq_small_box(small):
    g, o = small
    L = o.info()["L_eff"]
    B = int((0.5 * L - 1.0) / 0.5)   # largest range below L/2
    while (B - 1) * 0.5 + 1.0 >= 0.5 * L:
        B -= 1
    num, cnt = check_cq(g, o, 2 * math.pi / L * 6, 2 * math.pi / L * -1, 0.5, B)
    assert cnt[0] == 0 and cnt.sum() > 0   # no pair closer than sigma... nor 2 sigma
    assert np.all(np.abs(num) <= cnt + 1e-9)


def test_cq_medium_box_peak_and_accumulation(medium):
    g, o = medium
    N = MEDIUM["N"]
    L = o.info()["L_eff"]
    a0 = math.sqrt(2.0 / (math.sqrt(3.0) * N / L ** 2))
    qp = 4 * math.pi / (math.sqrt(3.0) * a0)
    h, k, _ = g.find_q0(0.9 * qp, 1.1 * qp, 0.0, math.pi / 3)
    qx, qy = 2 * math.pi / L * h, 2 * math.pi / L * k
    dr = 0.75   # a multiple of 2^-22; windows overlap (width 2 sigma)
    num, cnt = check_cq(g, o, qx, qy, dr, 70)
    # a second call adds the same configuration again
    num2, cnt2 = g.cq(qx, qy, dr, 70, num.copy(), cnt.copy())
    assert np.array_equal(cnt2, 2 * cnt)
    assert np.allclose(num2, 2 * num, rtol=0, atol=1e-9 * cnt.max())
    # at q = 0 every cosine is 1
    n0, c0 = g.cq(0.0, 0.0, dr, 70)
    assert np.array_equal(c0, cnt) and np.array_equal(n0, c0.astype(np.float64))


def test_cq_rejects_bad_windows(gpu_lib, small):
    g, o = small
    L = o.info()["L_eff"]
    for dr, B in ((0.1, 10), (0.5, 0), (0.5, 5000), (1.0, int(L / 2) + 2)):
        with pytest.raises(gpu_lib.MPMCError):
            g.cq(1.0, 0.0, dr, B)


def test_cq_aligned_matches_oracle_rotation(medium):
    """Psi_6 alignment: q turned by (arg Psi_6 - reference) / 6.  The GPU's
    Psi_6 is fp32 (1e-5 per disk), so its angle may differ from the oracle's
    by 2e-5 / (6 |Psi_6|) rad, and each cosine by |q| |d| times that."""
    g, o = medium
    L = o.info()["L_eff"]
    qx, qy = 2 * math.pi / L * 128, 2 * math.pi / L * 64
    Psi = o.psi6().mean()
    ref = np.angle(Psi) - 0.3          # as if the reference were turned by 0.05 rad
    a_o = math.remainder(np.angle(Psi) - ref, 2 * math.pi) / 6
    c, s = math.cos(a_o), math.sin(a_o)
    dr, B = 0.75, 40
    onum, ocnt = o.cq(c * qx - s * qy, s * qx + c * qy, dr, B)
    num, cnt, a = g.cq_aligned(qx, qy, ref, dr, B)
    da = 2e-5 / (6 * abs(Psi))
    assert abs(a - a_o) <= da and abs(a - 0.05) < 1e-12 + da
    assert np.array_equal(cnt, ocnt)
    top = (B - 1) * dr + 1
    assert np.all(np.abs(num - onum) <= ocnt * (math.hypot(qx, qy) * top * da + 1e-12))


def test_chi_right_after_sweeps(gpu_lib):
    """chi_j depends on absolute positions, hence on the accumulated shift
    that the sweeps advance on the device: a call straight after sweeps
    (nothing else read back in between) must see the current shift."""
    g = gpu_lib.Box(SMALL["N"], SMALL["eta"], seed=4, step_m=26, lattice="square")
    o = OracleBox(SMALL["N"], SMALL["eta"], seed=4, lattice=0, step_m=26)
    for k in (1, 7, 64):
        g.sweep(k)
        o.sweep(k)
        chi, _ = g.chi_field(5, -3)
        assert np.abs(chi - o.chi(5, -3)).max() < 1e-6
        S = g.structure_factor([[5, -3]])
        assert abs(S[0] - o.structure_factor([[5, -3]])[0]) <= s_tol(SMALL["N"], S[0])
