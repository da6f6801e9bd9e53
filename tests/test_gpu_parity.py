"""Parity of the HIP path with the CPU oracle, through the C ABI.

The plain sampler is compared bit for bit: cell lists (counts, tags, fp32
offsets in slot order), absolute positions, shifts and trial counters after
k sweeps.  Integer observables (contact counts) must be identical; psi_6 is
compared within 1e-5 per disk (fp32 on the GPU, fp64 in the oracle, same
neighbour sets).
"""
import math
import os

import numpy as np
import pytest

from oracle import orc
from oracle.orc import OracleBox

pytestmark = pytest.mark.gpu

SQUARE_256 = dict(N=256, eta=0.60, seed=0, lattice=0, step_m=26)
TRI_65536 = dict(N=65536, eta=0.716, seed=0, lattice=1, step_m=20)


def gpu_box(mp, N, eta, seed, lattice, step_m, n_trial=1, **kw):
    return mp.Box(N, eta, seed=seed, step_m=step_m, n_trial=n_trial,
                  lattice={0: "square", 1: "triangular", 2: "none"}[lattice], **kw)


def assert_same_state(g, o):
    gi, oi = g.info(), o.info()
    for k in ("sweep", "Sx", "Sy", "trials", "accepts", "M", "W"):
        assert gi[k] == oi[k], (k, gi[k], oi[k])
    gc, ocl = g.cells(), o.cells()
    names = ("cnt", "tag", "x", "y")
    for name, a, b in zip(names, gc, ocl):
        if a.dtype == np.float32:
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), name
        else:
            assert np.array_equal(a, b), name
    gX, gY = g.positions_q()
    oX, oY = o.positions_q()
    assert np.array_equal(gX, oX) and np.array_equal(gY, oY)


@pytest.mark.parametrize("schedule,tile,threads", [("simple", 0, 0), ("fused", 8, 64), ("fused", 8, 128)])
def test_n256_square_start_trajectory_bit_exact(gpu_lib, schedule, tile, threads):
    g = gpu_box(gpu_lib, **SQUARE_256, schedule="simple")
    g.set_schedule(schedule, tile, threads)
    o = OracleBox(**SQUARE_256)
    assert_same_state(g, o)
    done = 0
    for k in (1, 10, 100, 1000):
        g.sweep(k - done)
        o.sweep(k - done)
        done = k
        assert_same_state(g, o)
    assert g.validate() == (0, 0)


@pytest.mark.parametrize("n_trial", [2, 4])
def test_shuffled_trials_bit_exact(gpu_lib, n_trial):
    for schedule, tile in (("simple", 0), ("fused", 8)):
        g = gpu_box(gpu_lib, **SQUARE_256, n_trial=n_trial, schedule=schedule, tile=tile)
        o = OracleBox(**SQUARE_256, n_trial=n_trial)
        g.sweep(57)
        o.sweep(57)
        assert_same_state(g, o)


SPARSE = dict(N=64 * 64, eta=0.35, seed=3, lattice=0, step_m=200)


@pytest.mark.parametrize("tile,threads", [(8, 64), (24, 256), (34, 256), (48, 512)])
def test_fused_crowded_cells_bit_exact(gpu_lib, tile, threads):
    """Cells 2.8 sigma wide in a dilute box hold three disks now and then:
    the fused kernel tests slots 2 and 3 only in tiles that hold such a
    cell, and both forms must give the oracle's trajectory.  The 34- and
    48-cell tiles keep two slots per cell in LDS and slots 2 and 3 of such
    cells (11 to 21 of them per region here) in their side table."""
    g = gpu_box(gpu_lib, **SPARSE, cell_min=2.8, schedule="simple")
    g.set_schedule("fused", tile, threads)
    o = OracleBox(**SPARSE, cell_min=2.8)
    done = 0
    for k in (10, 100):
        g.sweep(k - done)
        o.sweep(k - done)
        done = k
        assert_same_state(g, o)
    assert (g.cells()[0] >= 3).sum() > 0
    assert g.validate() == (0, 0)


CROWDED = dict(N=72 * 72, eta=0.50, seed=5, lattice=0, step_m=200)


def crowded_per_region(cnt, side):
    """Cells of three or more disks in every side x side window of the
    periodic M x M grid (min, max over the windows)."""
    c = (cnt >= 3).astype(np.int64)
    M = c.shape[0]
    cc = np.pad(c, ((0, side), (0, side)), mode="wrap")
    S = np.pad(cc.cumsum(0).cumsum(1), ((1, 0), (1, 0)))
    v = S[side:M + side, side:M + side] - S[:M, side:M + side] - S[side:M + side, :M] + S[:M, :M]
    return int(v.min()), int(v.max())


@pytest.mark.parametrize("tile,threads", [(34, 256), (48, 512)])
def test_two_slot_tiles_with_more_crowded_cells_than_the_side_table(gpu_lib, tile, threads):
    """Cells 2.82 sigma wide at eta = 0.5 (M = 64): every tile region holds
    more than 32 cells of three or four disks, so every two-slot tile runs as
    four-slot sub-tiles; the trajectory is the oracle's."""
    g = gpu_box(gpu_lib, **CROWDED, cell_min=2.8, schedule="simple")
    g.set_schedule("fused", tile, threads)
    o = OracleBox(**CROWDED, cell_min=2.8)
    M = g.info()["M"]
    assert M == 64 and g.info()["w"] < 2.0 * math.sqrt(2.0)  # at most four disks a cell
    done = 0
    for k in (10, 100):
        g.sweep(k - done)
        o.sweep(k - done)
        done = k
        assert_same_state(g, o)
        assert crowded_per_region(g.cells()[0].reshape(M, M), tile + 9)[0] > 32
    assert g.validate() == (0, 0)


def test_two_slot_tiles_keep_every_disk_over_long_runs(gpu_lib):
    """N = 1024^2 at eta = 0.716 holds a few cells of three disks in most
    sweeps, so the 34-cell two-slot tile runs some tiles as four-slot
    sub-tiles in most launches.  Over 6000 sweeps the state stays valid
    (every tag once, offsets inside their cells, no overlap) and equals the
    four-slot 24-cell tile's trajectory bit for bit."""
    cfg = dict(N=1024 * 1024, eta=0.716, seed=4, lattice=1, step_m=55)
    a = gpu_box(gpu_lib, **cfg, schedule="fused", tile=34)
    b = gpu_box(gpu_lib, **cfg, schedule="fused", tile=24)
    for _ in range(6):
        a.sweep(1000)
        b.sweep(1000)
        assert a.validate() == (0, 0)
    for x, y in zip(a.cells(), b.cells()):
        assert np.array_equal(x, y)
    assert a.info()["trials"] == b.info()["trials"]


def test_n65536_triangular_trajectory_bit_exact(gpu_lib):
    g = gpu_box(gpu_lib, **TRI_65536)  # autotuned fused schedule
    assert g.info()["schedule"] == 2
    o = OracleBox(**TRI_65536)
    done = 0
    for k in (1, 10, 60, 1000):
        g.sweep(k - done)
        o.sweep(k - done)
        done = k
        assert_same_state(g, o)
    assert g.validate() == (0, 0)


def test_schedule_invariance_all_shapes(gpu_lib):
    """Every schedule (simple, each fused tile/threads shape, graphs on or
    off) gives the same trajectory."""
    ref = gpu_box(gpu_lib, **TRI_65536, schedule="simple")
    ref.sweep(20)
    rc = ref.cells()
    shapes = [(8, 64), (8, 128), (16, 128), (16, 256), (24, 256), (32, 256), (32, 512),
              (34, 256), (48, 512), (48, 1024)]
    for tile, threads in shapes:
        b = gpu_box(gpu_lib, **TRI_65536, schedule="simple")
        b.set_schedule("fused", tile, threads)
        b.set_graphs(0 if tile == 24 else 4)
        b.sweep(20)
        for a, c in zip(rc, b.cells()):
            assert np.array_equal(a, c), (tile, threads)


def test_graph_replay_matches_eager(gpu_lib):
    a = gpu_box(gpu_lib, **SQUARE_256, schedule="fused", tile=8)
    b = gpu_box(gpu_lib, **SQUARE_256, schedule="fused", tile=8)
    b.set_graphs(0)
    a.sweep(3)          # odd start: eager sweeps until the buffers line up
    a.sweep(300)        # graph replays of 128 sweeps
    a.sweep(1)
    for _ in range(304):
        b.sweep(1)
    for x, y in zip(a.cells(), b.cells()):
        assert np.array_equal(x, y)
    assert a.info()["trials"] == b.info()["trials"]


def test_checkpoint_resume_bit_exact(gpu_lib, tmp_path):
    a = gpu_box(gpu_lib, **SQUARE_256)
    a.sweep(50)
    a.accumulate_contacts()
    path = str(tmp_path / "ck.bin")
    a.save(path)
    a.sweep(70)
    b = gpu_lib.Box.load(path)
    b.sweep(70)
    for x, y in zip(a.cells(), b.cells()):
        assert np.array_equal(x, y)
    assert a.info()["sweep"] == b.info()["sweep"] == 120
    assert np.array_equal(a.contacts()[0], b.contacts()[0])


def test_contact_histogram_counts_identical(gpu_lib):
    g = gpu_box(gpu_lib, **SQUARE_256, hist_bins=20, hist_dr=0.01)
    o = OracleBox(**SQUARE_256)
    oc = np.zeros(20, np.int64)
    for _ in range(5):
        g.sweep(37)
        o.sweep(37)
        g.accumulate_contacts()
        o.pair_hist(20, 0.01, oc)
    gc, n = g.contacts()
    assert n == 5 and np.array_equal(gc, oc)
    res = g.measure_pressure()
    ref = orc.pressure_fit(oc, 0.01, 5, 256, o.info()["L_eff"])
    assert abs(res["P_star"] - ref["P_star"]) < 1e-10 * ref["P_star"]
    assert abs(res["g_contact"] - ref["g_contact"]) < 1e-10 * ref["g_contact"]


def test_contact_histogram_n65536_default_bins(gpu_lib):
    g = gpu_box(gpu_lib, **TRI_65536)
    o = OracleBox(**TRI_65536)
    g.sweep(30)
    o.sweep(30)
    g.accumulate_contacts()
    gc, _ = g.contacts()
    oc = o.pair_hist(100, 1e-3)
    assert np.array_equal(gc, oc)
    assert gc.sum() > 1000


def test_psi6_matches_oracle(gpu_lib):
    g = gpu_box(gpu_lib, **SQUARE_256)
    o = OracleBox(**SQUARE_256)
    g.sweep(200)
    o.sweep(200)
    psi, field, Psi = g.psi6_field()
    opsi = o.psi6()
    assert np.abs(psi - opsi).max() < 1e-5
    assert abs(Psi - opsi.mean()) < 1e-6
    ofield = o.psi6_field(opsi)
    assert np.abs(field - ofield).max() < 1e-5


def test_psi6_n65536_matches_oracle(gpu_lib):
    """Many 16 x 16 cell blocks (M = 226) of the tiled psi_6 kernel."""
    g = gpu_box(gpu_lib, **TRI_65536)
    o = OracleBox(**TRI_65536)
    g.sweep(40)
    o.sweep(40)
    psi, field, Psi = g.psi6_field()
    opsi = o.psi6()
    assert np.abs(psi - opsi).max() < 1e-5
    ofield = o.psi6_field(opsi)
    assert np.abs(field - ofield).max() < 1e-5


def test_fused_tiles_must_not_wrap(gpu_lib):
    """A tile whose halo region would cover the box twice is refused."""
    g = gpu_box(gpu_lib, **SQUARE_256, schedule="simple")
    with pytest.raises(gpu_lib.MPMCError):
        g.set_schedule("fused", 16, 256)   # 16 + 10 > M = 18


def test_n2_edge_case_bit_exact(gpu_lib):
    """Two disks in a 4 x 4 grid: the degenerate box (no fused tile fits)."""
    g = gpu_lib.Box(2, 0.05, seed=3, step_m=255, lattice="none")
    o = OracleBox(2, 0.05, seed=3, lattice=2, step_m=255)
    X = np.array([int(1.0 / orc.Q), int(5.5 / orc.Q)], np.int64)
    Y = np.array([int(1.0 / orc.Q), int(6.0 / orc.Q)], np.int64)
    g.set_positions_q(X, Y)
    o.set_positions_q(X, Y)
    assert g.info()["schedule"] == 1
    g.sweep(5000)
    o.sweep(5000)
    assert_same_state(g, o)


def test_full_size_parity_sampled(gpu_lib):
    """N = 1024^2 at eta = 0.716 in the benchmark's launch configuration:
    cell lists after 3 sweeps bit for bit, then sampled observables."""
    cfg = dict(N=1024 * 1024, eta=0.716, seed=0, lattice=1, step_m=20)
    g = gpu_box(gpu_lib, **cfg)
    o = OracleBox(**cfg)
    g.sweep(3)
    o.sweep(3)
    assert_same_state(g, o)
    rng = np.random.default_rng(0)
    sel = np.zeros(cfg["N"], np.uint8)
    sel[rng.choice(cfg["N"], 800, replace=False)] = 1
    assert np.array_equal(g.contact_hist_subset(sel), o.pair_hist_subset(sel, 100, 1e-3))
    psi, _, _ = g.psi6_field()
    opsi = o.psi6(sel)
    idx = np.nonzero(sel)[0]
    assert np.abs(psi[idx] - opsi[idx]).max() < 1e-5
    # positional order (Sec. IV.C): S at sampled wave vectors, chi sampled
    hk = np.array([[0, 0], [1, 0], [0, 1024], [-512, 886], [511, -886], [4095, 4095]], np.int32)
    S, So = g.structure_factor(hk), o.structure_factor(hk)
    assert np.all(np.abs(S - So) <= 2e-6 * np.sqrt(cfg["N"] * So) + 1e-12 * cfg["N"] + 1e-12)
    chi, _ = g.chi_field(-512, 886)
    assert np.abs(chi[idx] - o.chi(-512, 886)[idx]).max() < 1e-6
    # C_q at any size: at q = 0 every cosine is exactly 1; counts do not
    # depend on q; no pair is closer than 2 sigma
    n0, c0 = g.cq(0.0, 0.0, 0.5, 40)
    n1, c1 = g.cq(*g.wave_vector(-512, 886), 0.5, 40)
    assert np.array_equal(n0, c0.astype(np.float64)) and np.array_equal(c0, c1)
    assert c0[:2].sum() == 0 and c0[3] > 0 and np.all(np.abs(n1) <= c1)
    assert g.validate() == (0, 0)


@pytest.mark.parametrize("eta", [0.700, 0.720])
def test_paper_scale_densities_bit_exact(gpu_lib, eta):
    """N = 1024^2 at the ends of the paper's density scan (M = 1084 and 1068,
    a multiple of none of the tile sides, so the last tiles are ragged):
    cell lists after 2 sweeps bit for bit against the oracle."""
    cfg = dict(N=1024 * 1024, eta=eta, seed=1, lattice=1, step_m=20)
    g = gpu_box(gpu_lib, **cfg)
    o = OracleBox(**cfg)
    gi = g.info()
    assert gi["M"] == o.info()["M"] and gi["tile"] > 0 and gi["M"] % gi["tile"] != 0
    g.sweep(2)
    o.sweep(2)
    assert_same_state(g, o)
    assert g.validate() == (0, 0)


def test_largest_box_one_sweep_bit_exact(gpu_lib):
    """N = 4096^2 (M = 4288, 18.4 M cells, the state far beyond the Infinity
    Cache): cell lists and positions after one sweep bit for bit."""
    cfg = dict(N=4096 * 4096, eta=0.716, seed=2, lattice=1, step_m=20)
    g = gpu_box(gpu_lib, **cfg)
    o = OracleBox(**cfg)
    assert g.info()["M"] == 4288
    g.sweep(1)
    o.sweep(1)
    assert_same_state(g, o)


def test_gpu_n2_closed_form_pressure(gpu_lib):
    """Statistical pin of the GPU sampler itself: for N = 2 the separation is
    uniform outside the excluded disk, so P* = (4 eta/pi)(1-eta)/(1-2 eta)."""
    g = gpu_lib.Box(2, 0.05, seed=17, step_m=255, lattice="none", hist_bins=100, hist_dr=0.01,
                    hist_block=4000)
    X = np.array([int(1.0 / orc.Q), int(5.5 / orc.Q)], np.int64)
    Y = np.array([int(1.0 / orc.Q), int(6.0 / orc.Q)], np.int64)
    g.set_positions_q(X, Y)
    for _ in range(80000):
        g.sweep(3)
        g.accumulate_contacts()
    eta = g.info()["eta_eff"]
    res = g.measure_pressure()
    exact = 4 * eta / math.pi * (1 - eta) / (1 - 2 * eta)
    assert abs(res["P_star"] - exact) < 3 * res["se"], (res, exact)


def test_validate_counts_hand_placed_overlaps(gpu_lib):
    """mpmc_validate on hand-placed pairs: at 1.9 sigma, across the periodic
    edge at 1.06 sigma, at 2 - q (fp32 r^2 < 4), at exactly fp32 r^2 = 4
    (contact: no overlap) and a triple with two overlapping pairs: five
    overlaps, as the oracle counts them."""
    Q22 = 2 ** 22
    g = gpu_lib.Box(16, 0.008, seed=1, lattice="none", schedule="simple")
    Lq = g.info()["W"] * g.info()["M"]
    pts = [(10 * Q22, 10 * Q22), (10 * Q22 + int(1.9 * Q22), 10 * Q22),
           (Q22 // 2, 20 * Q22), (Lq - Q22 // 4, 20 * Q22 + 3 * Q22 // 4),
           (30 * Q22, 5 * Q22), (30 * Q22 + 2 * Q22 - 1, 5 * Q22),
           (5 * Q22, 30 * Q22), (5 * Q22, 32 * Q22),
           (20 * Q22, 30 * Q22), (21 * Q22, 30 * Q22), (22 * Q22 + Q22 // 2, 30 * Q22)]
    X = np.array([p[0] for p in pts] + [(40 + 5 * k) * Q22 for k in range(16 - len(pts))], np.int64)
    Y = np.array([p[1] for p in pts] + [40 * Q22] * (16 - len(pts)), np.int64)
    g.set_positions_q(X, Y)
    o = OracleBox(16, 0.008, lattice=2)
    o.set_positions_q(X, Y)
    assert o.count_overlaps() == 5
    assert g.validate() == (5, 0)
    # every pair but the contact one moved apart: no overlap remains
    for k in range(len(pts)):
        if k not in (6, 7):
            X[k], Y[k] = (10 + 5 * k) * Q22, 60 * Q22
    g.set_positions_q(X, Y)
    o.set_positions_q(X, Y)
    assert o.count_overlaps() == 0
    assert g.validate() == (0, 0)


def test_zero_length_calls_leave_the_state_alone(gpu_lib):
    """Empty requests: zero sweeps (plain and learned), zero wave vectors and
    zero contact accumulations leave the cell lists, the counters and the
    sweep index as they were."""
    g = gpu_lib.Box(4096, 0.70, seed=3, step_m=40, cell_min=3.0, schedule="simple")
    g.sweep(3)
    before = [c.copy() for c in g.cells()]
    i0 = g.info()
    assert g.sweep(0, counts=True) == (0, 0)
    L = gpu_lib.Learner(seed=1, capacity=16)
    assert gpu_lib.sweep_learned(g, L, 0, eps=0.1, counts=True) == (0, 0)
    assert len(g.structure_factor(np.zeros((0, 2), np.int32))) == 0
    i1 = g.info()
    for k in ("sweep", "trials", "accepts"):
        assert i1[k] == i0[k]
    for a, b in zip(before, g.cells()):
        assert np.array_equal(a, b)
    c, n = g.contacts()
    assert n == 0 and not c.any()


def test_upload_rejects_a_cell_beyond_capacity(gpu_lib):
    """More disks in one cell than its width can hold without overlap (the
    capacity the geometry derives) is refused on upload with MPMC_EOVERFLOW,
    before any kernel sees it, and the box keeps its state."""
    Q22 = 2 ** 22
    g = gpu_lib.Box(16, 0.008, seed=1, lattice="none", schedule="simple")
    info = g.info()
    cap, W, M = info["cap"], info["W"], info["M"]
    X = np.array([(10 + 4 * (k % 4)) * Q22 for k in range(16)], np.int64)
    Y = np.array([(10 + 4 * (k // 4)) * Q22 for k in range(16)], np.int64)
    g.set_positions_q(X, Y)
    before = [c.copy() for c in g.cells()]
    # cap + 1 disks spread inside cell (1, 1)
    for k in range(cap + 1):
        X[k] = W + (k * W) // (cap + 2)
        Y[k] = W + W // 2
    with pytest.raises(gpu_lib.MPMCError) as e:
        g.set_positions_q(X, Y)
    assert e.value.code == gpu_lib.EOVERFLOW
    for a, b in zip(before, g.cells()):
        assert np.array_equal(a, b)
    assert M > 2
