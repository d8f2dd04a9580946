"""dgn_step_noalloc (the allocation-free variant of dgn_step: the library's fixed
per-GPU scratch array is its workspace) against dgn_step with a context, through
the C ABI: two calls in a row, the second with a smaller input (the array keeps
the first call's contents, so anything that must start at zero is cleared by the
call), both bit-identical to dgn_step (the same kernels in the same order on the
same data); a shape beyond the array is rejected with DGN_ENOMEM."""
import numpy as np
import pytest
import torch

import cpgen

pytestmark = pytest.mark.gpu


def _dgn():
    from paper_1205_2584_amd import dgn
    return dgn


CASES = [((60, 50, 40), 12, torch.float32, 0.7), ((21, 18, 15, 6), 4, torch.float64, 0.2)]


def test_noalloc_step_matches_dgn_step():
    dgn = _dgn()
    ctx = dgn.Context(0, 1 << 28)
    for k, (dims, R, dt, mu) in enumerate(CASES):
        print(f"noalloc step {k}: dims={dims} R={R} dtype={dt}", flush=True)
        p = cpgen.small_problem(70 + k, dims, R, c=0.5, snr_db=25.0)
        y = torch.from_numpy(p.y).to(dt).cuda()
        need = dgn.workspace_size(dims, R, dt)
        assert need <= dgn.noalloc_scratch_bytes()
        ref, rinfo = ctx.dgn_step(y, dims, R, dgn.to_device_factors(p.init), mu)
        got, ginfo = dgn.dgn_step_noalloc(y, dims, R, dgn.to_device_factors(p.init), mu)
        for a, b in zip(dgn.to_host_factors(got), dgn.to_host_factors(ref)):
            assert np.array_equal(a, b)
        assert ginfo == rinfo
    ctx.close()


def test_noalloc_rejects_oversize():
    dgn = _dgn()
    dims, R = (100, 100, 100), 40
    assert dgn.workspace_size(dims, R, torch.float32) > dgn.noalloc_scratch_bytes()
    y = torch.zeros(int(np.prod(dims)), dtype=torch.float32, device="cuda")
    A = [torch.ones(R, I, dtype=torch.float64, device="cuda") for I in dims]
    with pytest.raises(dgn.DgnError) as e:
        dgn.dgn_step_noalloc(y, dims, R, A, 1.0)
    assert e.value.status == -2
    assert "scratch" in str(e.value)
