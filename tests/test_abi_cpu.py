"""Host-side checks of the C ABI that need no GPU: the library loads, every
symbol declared in include/mpmc.h is exported, parameters are validated
before any device work, and the host analysis (C(dt), tau) is right."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_1211_1645_amd import mpmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "mpmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return re.findall(r"^\s*(?:int|const char \*)\s*(mpmc_\w+)\s*\(", txt, re.M)


def test_library_exports_every_declared_symbol():
    lib = mpmc.load()
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps every declared entry point
    assert set(names) - {"mpmc_last_error"} <= set(mpmc._SIGS)


def test_default_params():
    lib = mpmc.load()
    p = mpmc.Params()
    assert lib.mpmc_default_params(C.byref(p)) == 0
    assert (p.step_m, p.n_trial, p.lattice, p.hist_bins, p.fit_order) == (26, 1, 1, 100, 4)
    assert p.cell_min == 2.0 and p.hist_dr == 1e-3
    assert lib.mpmc_default_params(None) == mpmc.EINVAL


@pytest.mark.parametrize("N,eta,kw,frag", [
    (0, 0.5, {}, "N must be positive"),
    (256, 0.0, {}, "eta"),
    (256, 0.8, {}, "eta"),
    (4, 0.5, {}, "box too small"),
    (255, 0.5, {}, "perfect square"),
    (256, 0.6, {"step_m": 0}, "step_m"),
    (256, 0.6, {"n_trial": 0}, "n_trial"),
    (256, 0.6, {"hist_bins": 5000}, "hist_bins"),
    (256, 0.6, {"hist_dr": 0.1}, "below r = 4"),
    (256, 0.6, {"fit_order": 0}, "fit_order"),
    (256, 0.6, {"schedule": 7}, "schedule"),
])
def test_invalid_parameters_rejected_before_device_work(N, eta, kw, frag):
    lib = mpmc.load()
    p = mpmc.Params()
    lib.mpmc_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    h = C.c_void_p()
    rc = lib.mpmc_init_box(C.byref(h), N, eta, 0, C.byref(p))
    assert rc == mpmc.EINVAL
    assert frag in lib.mpmc_last_error().decode()
    assert not h.value


def test_null_handles():
    lib = mpmc.load()
    assert lib.mpmc_free_box(None) == 0
    assert lib.mpmc_sweep(None, 1, None, None) == mpmc.EINVAL
    assert lib.mpmc_measure_pressure(None, None, None, None, None) == mpmc.EINVAL
    assert lib.mpmc_init_box(None, 256, 0.6, 0, None) == mpmc.EINVAL
    assert lib.mpmc_structure_factor(None, None, 1, None) == mpmc.EINVAL
    assert lib.mpmc_find_q0(None, 1.0, 2.0, 0.0, 1.0, None, None, None) == mpmc.EINVAL
    assert lib.mpmc_chi_field(None, 1, 0, None, None, None, None, 0) == mpmc.EINVAL
    assert lib.mpmc_cq(None, 1.0, 0.0, 0.5, 4, None, None) == mpmc.EINVAL


def test_acf_and_tau_on_ar1():
    """Host analysis of Eq. (9): an AR(1) series Psi(t+1) = phi Psi(t) + noise
    has C(dt) = phi^dt and tau = -1/ln(phi)."""
    rng = np.random.default_rng(1)
    phi, n = 0.9, 300000
    e = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    s = np.empty(n, complex)
    s[0] = e[0]
    for t in range(1, n):
        s[t] = phi * s[t - 1] + e[t]
    Cv = mpmc.acf(s, 120)
    assert np.allclose(Cv[:40], phi ** np.arange(40), atol=0.02)
    tau, tau_int = mpmc.tau(Cv)
    exact = -1 / math.log(phi)
    assert abs(tau - exact) / exact < 0.05
    assert abs(tau_int - (1 + phi) / (2 * (1 - phi))) / ((1 + phi) / (2 * (1 - phi))) < 0.1
    # agrees with the oracle's estimator
    from oracle import orc
    assert np.allclose(Cv, orc.acf(s, 120), rtol=1e-10, atol=1e-12)


def test_tau_rejects_short_window():
    with pytest.raises(mpmc.MPMCError):
        mpmc.tau(np.array([1.0, 0.01, 0.0, 0.0]))


def test_cq_bin_max_groups():
    """Incoherent averaging takes the maximum within groups of windows; the
    last group may be short."""
    rng = np.random.default_rng(4)
    c = rng.normal(size=23)
    out = mpmc.cq_bin_max(c, 5)
    want = [c[i:i + 5].max() for i in range(0, 23, 5)]
    assert np.array_equal(out, want)
    assert np.array_equal(mpmc.cq_bin_max(c, 1), c)
    assert mpmc.load().mpmc_cq_bin_max(None, 3, 1, None) == mpmc.EINVAL
