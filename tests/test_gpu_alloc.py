"""The device allocator hook of mpmc_params: a box whose memory comes from
torch's caching allocator runs the same trajectory as one using hipMalloc,
and a hook that fails makes mpmc_init_box return MPMC_ENOMEM after handing
back every allocation it had made."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_torch_allocator_same_trajectory(gpu_lib):
    a = gpu_lib.Box(64 * 64, 0.70, seed=3, step_m=40, torch_allocator=True)
    b = gpu_lib.Box(64 * 64, 0.70, seed=3, step_m=40)
    for k in (1, 37, 200):
        a.sweep(k)
        b.sweep(k)
        for u, v in zip(a.cells(), b.cells()):
            assert np.array_equal(u, v)
    for box in (a, b):
        box.accumulate_contacts()
    assert np.array_equal(a.contacts()[0], b.contacts()[0])
    psi_a, _, Psi_a = a.psi6_field()
    psi_b, _, Psi_b = b.psi6_field()
    assert np.array_equal(psi_a, psi_b) and Psi_a == Psi_b
    assert a.validate() == (0, 0)


@pytest.mark.parametrize("fail_at", [0, 1, 3, 6])
def test_failing_allocator_gives_enomem_and_frees(gpu_lib, fail_at):
    import torch
    lib = gpu_lib.load()
    p = gpu_lib.Params()
    assert lib.mpmc_default_params(C.byref(p)) == 0
    live, log = {}, {"allocs": 0, "frees": 0}

    def alloc(n, ctx):
        if log["allocs"] >= fail_at:
            return None
        log["allocs"] += 1
        ptr = torch.cuda.caching_allocator_alloc(int(n))
        live[ptr] = n
        return ptr

    def free(ptr, ctx):
        log["frees"] += 1
        live.pop(ptr)
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = gpu_lib._alloc_t(alloc), gpu_lib._free_t(free)
    p.alloc, p.free = fa, ff
    h = C.c_void_p()
    rc = lib.mpmc_init_box(C.byref(h), 64 * 64, 0.70, 1, C.byref(p))
    assert rc == gpu_lib.ENOMEM, (rc, lib.mpmc_last_error())
    assert not h.value
    assert log["allocs"] == fail_at and log["frees"] == fail_at and not live
