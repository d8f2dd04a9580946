"""The device-side problem generator builds the same CP tensor as the host one."""
import numpy as np
import pytest
import torch

import cpgen
from cpgen import device as cdev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("dims", [(5, 4, 3), (6, 5, 4, 3), (3, 4, 2, 2, 3)])
def test_cp_tensor_device_matches_host(dims, complex_):
    rng = np.random.default_rng(len(dims))
    R = 3
    A = [rng.standard_normal((I, R)) + (1j * rng.standard_normal((I, R)) if complex_ else 0) for I in dims]
    ref = cpgen.cp_tensor(A)
    got = cdev.cp_tensor_device(torch, [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in A])
    assert np.linalg.norm(got.cpu().numpy() - ref) <= 1e-13 * np.linalg.norm(ref)


def test_pool_shapes_and_snr():
    pool = cdev.make_pool(torch, 7, 6, imax=40, max_elems=1 << 16)
    for p in pool:
        assert 3 <= len(p.dims) <= 4 and all(16 <= I <= 40 for I in p.dims) and 2 <= p.R <= 20
        assert p.y.numel() == int(np.prod(p.dims))
        assert p.y.dtype == (torch.complex64 if p.complex_ else torch.float32)
        assert all(a.shape == (I, p.R) for a, I in zip(p.init, p.dims))
