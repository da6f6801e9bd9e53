"""Host-side pieces of bench.py that need no GPU: the correlation-time
analysis of a Psi_6 series and the stored-profile readers."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_tau_analysis_on_ar1_series():
    """A complex AR(1) series Psi(t+1) = phi Psi(t) + noise has C(dt) = phi^dt:
    tau = -1/ln(phi) samples and the e-folding lag is its ceiling."""
    rng = np.random.default_rng(3)
    phi, n = 0.98, 100000
    noise = rng.normal(size=n) + 1j * rng.normal(size=n)
    x = np.empty(n, np.complex128)
    x[0] = noise[0]
    for t in range(1, n):
        x[t] = phi * x[t - 1] + noise[t]
    sample, disp = 10, 0.5   # sweeps per sample, displacements per disk per sweep
    res = bench.tau_analysis(x, sample, disp, discard=1000 * sample)
    tau_s = -1.0 / math.log(phi)   # in samples
    unit = sample * disp
    # the e-folding lag and the integrated time are tight at 2000 tau; the
    # exponential fit over 0.05 <= C <= 0.5 leans on the noisy tail
    assert res["tau_efold_displacements_per_disk"] == pytest.approx(tau_s * unit, rel=0.08)
    assert res["tau_int_displacements_per_disk"] == pytest.approx(tau_s * unit, rel=0.1)
    assert res["tau_displacements_per_disk"] == pytest.approx(tau_s * unit, rel=0.3)
    assert res["tau_sweeps"] == pytest.approx(res["tau_displacements_per_disk"] / disp)
    for h in res["tau_efold_halves_displacements_per_disk"]:
        assert h == pytest.approx(tau_s * unit, rel=0.12)


def test_stored_profiles_are_readable():
    tau = bench.stored_tau()
    assert tau is not None and tau["paper_tau_displacements_per_disk"] == 8.0e5
    assert tau["tau_efold_displacements_per_disk"] > 0
    # the traffic figure is reported only for the kernel source it was taken on
    t = bench.stored_traffic()
    assert t is None or t > bench.algorithmic_bytes_per_sweep(1024 * 1024, 1072)


def test_stored_pressure_agrees_with_table_one():
    """The committed pressure run at N = 256^2, eta = 0.698 against the
    paper's MPMC value (Table I): its own replica error, recomputed from the
    stored replica means, and agreement within three combined errors."""
    import json
    import math
    import os
    p = bench.stored_pressure()
    assert p is not None and p["paper_p_star"] == 9.17078 and p["replicas"] >= 8
    d = json.load(open(os.path.join(bench.ROOT, p["source"])))
    rep = d["replica_means"]
    mean = sum(rep) / len(rep)
    sd = math.sqrt(sum((x - mean) ** 2 for x in rep) / (len(rep) - 1))
    assert mean == pytest.approx(p["p_star"], abs=1e-12)
    assert sd / math.sqrt(len(rep)) == pytest.approx(p["se"], rel=1e-9)
    assert abs(p["p_star"] - 9.17078) < 3 * math.hypot(p["se"], 4.5e-5)


def test_stored_tau_compare_is_consistent():
    """The committed learned-against-plain comparison: each rate is the
    run's sweeps per second over its tau in sweeps, and the reported gains
    are the ratios of those figures."""
    import json
    import os
    c = bench.stored_tau_compare()
    assert c is not None and c["provenance"].startswith("stored")
    assert set(c["decorrelations_per_s"]) == {"plain_w3", "plain_w2_fused", "learned_w3"}
    d = json.load(open(os.path.join(bench.ROOT, "profiles",
                                    "psi6_tau_learned_vs_plain_128sq_eta066.json")))
    s = d["samplers"]
    for k, v in s.items():
        assert v["decorrelations_per_s"] == pytest.approx(v["sweeps_per_s"] / v["tau_sweeps"], rel=1e-9)
        assert c["tau_sweeps"][k] == [v["tau_sweeps"], v["tau_sweeps_se"]]
    rate = {k: v["decorrelations_per_s"] for k, v in s.items()}
    assert c["gain_decorrelations_per_s_vs_plain_w3"] == pytest.approx(
        rate["learned_w3"] / rate["plain_w3"], rel=1e-9)
    assert c["gain_decorrelations_per_s_vs_plain_w2_fused"] == pytest.approx(
        rate["learned_w3"] / rate["plain_w2_fused"], rel=1e-9)
    assert c["gain_tau_per_sweep_vs_plain_w3"] == pytest.approx(
        s["plain_w3"]["tau_sweeps"] / s["learned_w3"]["tau_sweeps"], rel=1e-9)


class _StubBox:
    def __init__(self, w):
        self.w = w

    def info(self):
        return {"w": self.w}


def test_max_step_keeps_width_plus_step_below_four():
    """The step m moves a disk by at most m/256 sigma per coordinate; the
    largest m the box allows keeps w + m/256 below 4 sigma, capped at 255."""
    for w in (2.0, 2.5, 3.0, 3.04, 3.5, 3.66, 3.99):
        m = bench.max_step(_StubBox(w))
        assert 0 <= m <= 255
        assert w + m / 256.0 < 4.0
        assert m == 255 or w + (m + 1) / 256.0 >= 4.0
