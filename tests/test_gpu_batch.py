"""Batched boxes: every box of a batch evolves bit for bit as the same box
run alone (and as the oracle), whatever the tile schedule."""
import numpy as np
import pytest

from oracle.orc import OracleBox
from paper_1211_1645_amd.workloads import batch_boxes

pytestmark = pytest.mark.gpu


def same_cells(a, b):
    for x, y in zip(a.cells(), b.cells()):
        if not np.array_equal(x, y):
            return False
    return True


def test_batch_matches_single_boxes(gpu_lib):
    N = [16 ** 2, 24 ** 2, 32 ** 2, 40 ** 2, 64 ** 2, 20 ** 2]
    eta = [0.70, 0.65, 0.72, 0.69, 0.716, 0.5]
    seed = [3, 4, 5, 6, 7, 8]
    bt = gpu_lib.Batch(N, eta, seed, step_m=30)
    info = bt.info()
    assert info["nbox"] == 6
    bt.set_graphs(16)
    bt.sweep(3)
    bt.sweep(40)
    for i in range(6):
        single = gpu_lib.Box(N[i], eta[i], seed=seed[i], step_m=30, schedule="simple")
        single.sweep(43)
        assert same_cells(bt.box(i), single), i
        assert bt.box(i).info()["trials"] == single.info()["trials"]
    # and against the oracle for one of them
    o = OracleBox(N[1], eta[1], seed=seed[1], lattice=1, step_m=30)
    o.sweep(43)
    for x, y in zip(bt.box(1).cells(), o.cells()):
        assert np.array_equal(x, y)


def test_batch_schedules_agree(gpu_lib):
    N, eta, seed = batch_boxes(nbox=8, seed=1, sides=(64, 96))
    ref = gpu_lib.Batch(N, eta, seed, step_m=40)
    ref.set_schedule(0, 1)  # per-box simple kernels
    ref.sweep(12)
    for tile, threads in [(8, 128), (24, 256), (34, 256), (48, 512)]:
        bt = gpu_lib.Batch(N, eta, seed, step_m=40)
        bt.set_schedule(tile, threads)
        bt.sweep(12)
        for i in range(len(N)):
            assert same_cells(bt.box(i), ref.box(i)), (tile, threads, i)


def test_batch_of_64_uneven_boxes(gpu_lib):
    N, eta, seed = batch_boxes(nbox=64, seed=0)
    bt = gpu_lib.Batch(N, eta, seed, step_m=40, hist_bins=100, hist_dr=1e-3)
    info = bt.info()
    assert info["tile"] > 0 and info["n_items"] > 64
    t, a = bt.sweep(64, counts=True)
    assert t > 0 and 0.05 < a / t < 0.95
    bt.accumulate_contacts()
    P, se = bt.measure_pressure()
    assert (P > 5).all() and (P < 20).all()
    for i in (0, 37, 63):
        b = bt.box(i)
        assert b.validate() == (0, 0)
        single = gpu_lib.Box(int(N[i]), float(eta[i]), seed=int(seed[i]), step_m=40)
        single.sweep(64)
        assert same_cells(b, single)
    with pytest.raises(gpu_lib.MPMCError):
        bt.box(0).sweep(1)  # batch members are swept by the batch only


def test_autotune_choice_kept_in_file(gpu_lib, tmp_path, monkeypatch):
    """With MPMC_TUNE_CACHE naming a file, a tuned choice is appended to it,
    and a line for another grid is taken instead of tuning that grid; the
    shape never changes the trajectory."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MPMC_TUNE_CACHE", str(path))
    a = gpu_lib.Box(144 * 144, 0.70, seed=1, step_m=30, n_trial=2)
    ia = a.info()
    lines = [l for l in path.read_text().splitlines() if l.strip()]
    assert len(lines) == 1
    f = lines[0].split()
    assert (int(f[2]), int(f[3]), int(f[4])) == (ia["M"], 2, ia["tile"])
    Mb = gpu_lib.Box(172 * 172, 0.70, seed=1, step_m=30, n_trial=2, schedule="simple").info()["M"]
    assert Mb != ia["M"]
    path.write_text(lines[0] + "\n" + "%s %s %d 2 8 64\n" % (f[0], f[1], Mb))
    b = gpu_lib.Box(172 * 172, 0.70, seed=1, step_m=30, n_trial=2)
    assert b.info()["tile"] == 8
    assert len([l for l in path.read_text().splitlines() if l.strip()]) == 2  # nothing tuned
    c = gpu_lib.Box(172 * 172, 0.70, seed=1, step_m=30, n_trial=2, schedule="fused", tile=24)
    b.sweep(10)
    c.sweep(10)
    for x, y in zip(b.cells(), c.cells()):
        assert np.array_equal(x, y)
