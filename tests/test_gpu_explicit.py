"""dgn_step_explicit (the plain dGN step of Section 3 with J^T J formed
explicitly, the paper's comparison baseline) against the oracle's
explicit-Jacobian step, and against the fast step dgn_step: Theorem 4.1 makes
the two steps the same vector, so they may differ only by rounding.

Tolerance: both GPU steps and the oracle solve a positive definite system
(J^T J + mu I) in FP64; at the mu used here its condition number stays below
1e5, so 1e-9 relative leaves a wide margin over the rounding of either solve.
"""
import numpy as np
import pytest
import torch

import cpgen
from oracle import brute, cp

pytestmark = pytest.mark.gpu


def _dgn():
    from paper_1205_2584_amd import dgn
    return dgn


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dims,R,mu", [((8, 7, 6), 1, 1.0), ((9, 8, 7), 3, 0.5), ((6, 5, 4, 3), 2, 2.0),
                                       ((20, 18, 16), 6, 1.0), ((12, 10, 9, 7), 4, 10.0)])
def test_explicit_step_matches_oracle(dims, R, mu):
    dgn = _dgn()
    p = cpgen.small_problem(700 + R, dims, R, c=0.5, snr_db=20.0)
    dref, _, _ = brute.plain_step(p.y, p.init, mu)
    y = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size_explicit(dims, R) + (16 << 20))
    try:
        A = dgn.to_device_factors(p.init)
        out, info = ctx.dgn_step_explicit(y, dims, R, A, mu)
        got = [a - b for a, b in zip(dgn.to_host_factors(out), p.init)]
    finally:
        ctx.close()
    for g, w in zip(got, dref):
        assert _rel(g, w) < 1e-9
    Y = cp.as_tensor(p.y, dims)
    assert abs(info["err2_old"] - cp.residual_norm2(Y, p.init)) <= 1e-10 * info["err2_old"]
    new = [a + d for a, d in zip(p.init, dref)]
    assert abs(info["err2_new"] - cp.residual_norm2(Y, new)) <= 1e-9 * info["err2_old"]


@pytest.mark.parametrize("dims,R,mu", [((40, 35, 30), 8, 5.0), ((100, 100, 100), 20, 50.0), ((20, 18, 16, 14), 5, 2.0)])
def test_explicit_step_equals_fast_step(dims, R, mu):
    dgn = _dgn()
    p = cpgen.small_problem(730 + R, dims, R, c=0.7, snr_db=25.0)
    y = torch.from_numpy(p.y).cuda()
    ws = max(dgn.workspace_size_explicit(dims, R), dgn.workspace_size(dims, R)) + (16 << 20)
    ctx = dgn.Context(0, ws)
    try:
        A = dgn.to_device_factors(p.init)
        oe, ie = ctx.dgn_step_explicit(y, dims, R, A, mu)
        of, if_ = ctx.dgn_step(y, dims, R, A, mu)
        de = [a - b for a, b in zip(dgn.to_host_factors(oe), p.init)]
        df = [a - b for a, b in zip(dgn.to_host_factors(of), p.init)]
    finally:
        ctx.close()
    for a, b in zip(de, df):
        assert _rel(a, b) < 1e-9
    assert ie["err2_old"] == if_["err2_old"]  # same pass and error kernels
    for k in ("err2_new", "denom", "gnorm", "danorm"):
        assert abs(ie[k] - if_[k]) <= 1e-9 * abs(if_[k])


def test_explicit_step_rejects_complex():
    dgn = _dgn()
    dims, R = (6, 5, 4), 2
    ctx = dgn.Context(0, 64 << 20)
    try:
        y = torch.zeros(int(np.prod(dims)), dtype=torch.complex128, device="cuda")
        A = [torch.zeros((R, I), dtype=torch.complex128, device="cuda") for I in dims]
        with pytest.raises(dgn.DgnError) as e:
            ctx.dgn_step_explicit(y, dims, R, A, 1.0)
        assert e.value.status == -1
    finally:
        ctx.close()
