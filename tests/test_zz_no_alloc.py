"""The allocation-free structure factor against the allocating entry point:
same kernels, same partial layout and reduction, so the values agree bit
for bit; two calls in a row, the second smaller, then the limits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_structure_factor_noalloc_matches(gpu_lib):
    import torch
    box = gpu_lib.Box(64 * 64, 0.70, seed=3, step_m=40)
    box.sweep(20)
    rng = np.random.default_rng(1)
    for nq in (3000, 37):
        hk = rng.integers(-200, 200, size=(nq, 2)).astype(np.int32)
        ref = box.structure_factor(hk)
        hk_d = torch.from_numpy(hk).cuda()
        S_d = torch.full((nq,), -1.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        box.structure_factor_noalloc(hk_d, S_d)
        torch.cuda.synchronize()
        got = S_d.cpu().numpy()
        assert np.array_equal(got, ref), (nq, np.abs(got - ref).max())
        box.sweep(5)
    # the limits: more wave vectors than the scratch holds; an index outside
    # the stated range gives NaN in its entry only
    hk_big = torch.zeros((4097, 2), dtype=torch.int32, device="cuda")
    S_big = torch.zeros(4097, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.MPMCError) as e:
        box.structure_factor_noalloc(hk_big, S_big)
    assert e.value.code == gpu_lib.EINVAL
    hk = np.array([[1, 0], [4096, 0], [0, 2]], np.int32)
    S_d = torch.zeros(3, dtype=torch.float64, device="cuda")
    box.structure_factor_noalloc(torch.from_numpy(hk).cuda(), S_d)
    torch.cuda.synchronize()
    got = S_d.cpu().numpy()
    assert np.isnan(got[1]) and np.isfinite(got[[0, 2]]).all()
    assert np.array_equal(got[[0, 2]], box.structure_factor(hk[[0, 2]]))
