"""Asynchronous measurement (contact histogram and psi_6 on the box's own
stream, overlapping the following sweeps) against the synchronous calls on
an identical box: the same Psi_6 series, contact counts and pressure, bit
for bit, and the sampler state unaffected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CFG = dict(N=65536, eta=0.716, seed=0)


def make(mp, graphs):
    b = mp.Box(CFG["N"], CFG["eta"], seed=CFG["seed"], step_m=20, lattice="triangular",
               schedule="fused", tile=24)
    b.set_graphs(graphs)
    return b


@pytest.mark.parametrize("graphs,per_step", [(10, 10), (0, 3), (32, 33)])
def test_async_matches_sync(gpu_lib, graphs, per_step):
    import torch
    a, s = make(gpu_lib, graphs), make(gpu_lib, graphs)
    steps = 6
    psi_dev = torch.zeros(steps, 2, dtype=torch.float64, device="cuda")
    psi_sync = []
    for k in range(steps):
        a.sweep(per_step)
        a.measure_async(psi_dev[k], field=(k % 2 == 0))
        s.sweep(per_step)
        s.accumulate_contacts()
        _, _, P = s.psi6_field()
        psi_sync.append(P)
    assert a.measure_wait() is False
    got = psi_dev.cpu().numpy()
    want = np.array([[p.real, p.imag] for p in psi_sync])
    assert np.array_equal(got, want)
    ca, na = a.contacts()
    cs, ns = s.contacts()
    assert na == ns == steps and np.array_equal(ca, cs)
    assert a.measure_pressure()["P_star"] == s.measure_pressure()["P_star"]
    for x, y in zip(a.cells(), s.cells()):
        assert np.array_equal(x, y)
    assert a.info()["sweep"] == s.info()["sweep"] == steps * per_step


def test_async_rejects_pressure_blocks(gpu_lib):
    b = gpu_lib.Box(4096, 0.7, seed=1, step_m=20, hist_block=10)
    with pytest.raises(gpu_lib.MPMCError):
        b.measure_async()


def test_async_wider_search_runs_on_device(gpu_lib):
    """At eta = 0.5 some disks have their sixth neighbour beyond the two cells
    of the first psi_6 pass (checked here from the box's own positions), so
    the device-gated second pass must run: the asynchronous Psi_6 still
    equals the synchronous one bit for bit and no failure is reported."""
    import torch
    kw = dict(step_m=40, lattice="triangular")
    a = gpu_lib.Box(4096, 0.5, seed=0, **kw)
    s = gpu_lib.Box(4096, 0.5, seed=0, **kw)
    a.sweep(200)
    s.sweep(200)
    info = a.info()
    x, y = a.positions()
    L, w = info["M"] * info["w"], info["w"]
    d6 = np.empty(len(x))
    for i in range(0, len(x), 512):
        dx = x[i:i + 512, None] - x[None, :]
        dx -= L * np.round(dx / L)
        dy = y[i:i + 512, None] - y[None, :]
        dy -= L * np.round(dy / L)
        d6[i:i + 512] = np.sort(np.hypot(dx, dy), axis=1)[:, 6]
    assert (d6 > 2 * w).any() and (d6 < 3 * w).all()
    psi = torch.zeros(2, dtype=torch.float64, device="cuda")
    a.measure_async(psi, field=True)
    assert a.measure_wait() is False
    _, _, P = s.psi6_field()
    assert psi[0].item() == P.real and psi[1].item() == P.imag


def test_async_reports_search_too_short(gpu_lib):
    """At eta = 0.15, after the lattice has dissolved, the sixth neighbour of
    most disks lies beyond three cells, the widest staged stencil: the
    asynchronous measurement cannot retry further and must say so, once."""
    b = gpu_lib.Box(4096, 0.15, seed=0, step_m=255, lattice="triangular")
    b.sweep(300)
    b.measure_async()
    assert b.measure_wait() is True
    assert b.measure_wait() is False
    b.measure_async()
    assert b.measure_wait() is True
