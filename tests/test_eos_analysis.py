"""Equation-of-state loop analysis (Sec. IV.A): the numpy oracle pinned by a
closed form, and the library's host implementation against the oracle.

Synthetic equations of state: P*(v) = P_c + k (v - v0)((v - v0)^2 - d^2) in
the area per disk v = pi / eta, with its extrema at eta = 0.702 and 0.714 (the
loop positions the paper reports for large boxes) around P* = 9.15, the loop
height shrinking with N, plus Gaussian noise of a stated standard error.
"""
import math

import numpy as np
import pytest

from oracle import eos
from paper_1211_1645_amd import mpmc

ETA_A, ETA_B, PC = 0.702, 0.714, 9.15


def cubic_loop(k, eta):
    va, vb = math.pi / ETA_A, math.pi / ETA_B
    v0 = 0.5 * (va + vb)
    d = (va - v0) * math.sqrt(3.0)
    v = math.pi / np.asarray(eta)
    return PC + k * (v - v0) * ((v - v0) ** 2 - d * d), v0, d


def closed_form(k):
    _, v0, d = cubic_loop(k, [0.7])
    return dict(eta_max=ETA_A, eta_min=ETA_B, P_coex=PC, eta_liquid=math.pi / (v0 + d),
                eta_solid=math.pi / (v0 - d), delta_f=0.25 * abs(k) * d ** 4 / 4)


ETA = np.linspace(0.69, 0.73, 41)


def test_oracle_cubic_closed_form():
    """An odd cubic about v0 has the Maxwell line through its centre, roots at
    v0 and v0 +- d, extrema at v0 +- d/sqrt(3), and one lobe of area k d^4/4."""
    for k in (-40.0, -5.0):
        P, _, _ = cubic_loop(k, ETA)
        r = eos.loop(ETA, P, 3)
        want = closed_form(k)
        for key, val in want.items():
            assert r[key] == pytest.approx(val, rel=1e-10, abs=1e-14), key


def test_oracle_no_loop_and_power_law():
    assert eos.loop(ETA, 5.0 + 20.0 * ETA, 3) is None      # monotone
    N = np.array([256.0 ** 2, 512.0 ** 2, 1024.0 ** 2])
    b, a = eos.power_law(N, 3.0 * N ** -0.5)
    assert b == pytest.approx(-0.5, abs=1e-12) and a == pytest.approx(3.0, rel=1e-10)


def test_library_closed_form():
    for k in (-40.0, -5.0):
        P, _, _ = cubic_loop(k, ETA)
        r = mpmc.eos_loop(ETA, P, order=3)
        want = closed_form(k)
        assert r["p_coex"] == pytest.approx(want["P_coex"], rel=1e-12)
        for key in ("eta_max", "eta_min", "eta_liquid", "eta_solid", "delta_f"):
            assert r[key] == pytest.approx(want[key], rel=1e-9), key


@pytest.mark.parametrize("seed,order,weighted", [(0, 3, False), (1, 3, True), (2, 5, False),
                                                 (3, 5, True), (4, 4, True)])
def test_library_matches_oracle_on_noisy_data(seed, order, weighted):
    rng = np.random.default_rng(seed)
    se = rng.uniform(0.002, 0.006, ETA.size)
    P, _, _ = cubic_loop(-40.0, ETA)
    P = P + rng.normal(0.0, 1.0, ETA.size) * se
    o = eos.loop(ETA, P, order, se if weighted else None)
    if o is None:
        with pytest.raises(mpmc.MPMCError):
            mpmc.eos_loop(ETA, P, se if weighted else None, order)
        return
    g = mpmc.eos_loop(ETA, P, se if weighted else None, order)
    assert g["p_coex"] == pytest.approx(o["P_coex"], rel=1e-10)
    for key, okey in (("eta_max", "eta_max"), ("eta_min", "eta_min"), ("p_max", "P_max"),
                      ("p_min", "P_min"), ("eta_liquid", "eta_liquid"),
                      ("eta_solid", "eta_solid")):
        assert g[key] == pytest.approx(o[okey], rel=1e-8), key
    assert g["delta_f"] == pytest.approx(o["delta_f"], rel=1e-6)


def test_library_rejects_and_scales():
    with pytest.raises(mpmc.MPMCError):
        mpmc.eos_loop(ETA, 5.0 + 20.0 * ETA)               # no loop
    with pytest.raises(mpmc.MPMCError):
        mpmc.eos_loop(ETA[:4], ETA[:4])                    # too few points
    with pytest.raises(mpmc.MPMCError):
        mpmc.eos_loop(ETA, ETA, order=2)
    # loops of three box sizes whose height shrinks as N^-1/2: Delta f too
    N = np.array([256.0 ** 2, 512.0 ** 2, 1024.0 ** 2])
    df = []
    for n in N:
        P, _, _ = cubic_loop(-40.0 * 256.0 / math.sqrt(n), ETA)
        df.append(mpmc.eos_loop(ETA, P)["delta_f"])
    b, a = mpmc.power_law(N, df)
    ob, oa = eos.power_law(N, df)
    assert b == pytest.approx(-0.5, abs=1e-9) and b == pytest.approx(ob, abs=1e-12)
    assert a == pytest.approx(oa, rel=1e-10)
    with pytest.raises(mpmc.MPMCError):
        mpmc.power_law([1.0, 1.0], [2.0, 3.0])
