"""dgn_hessian_solve: (J^T J + mu I)^-1 v for any v, the inverse of H_mu in the
block form of Section 4.1, against the explicit-Jacobian solve of the oracle
(oracle/brute.py: J formed entry by entry, numpy.linalg.solve).

Tolerance: both sides solve the same SPD system in FP64; the GPU's result
differs by rounding amplified by cond(J^T J + mu I), which the cases keep
below about 1e4, so 1e-9 relative leaves three orders of margin (the same bar
as the step parity).  With the iterative solve (tolerance 1e-12) the bound is
10 cond(S) 1e-12 on top, computed as in tests/test_gpu_cg.py.
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


CASES = [((12, 10, 9), 3, 1.0), ((8, 7, 6, 5), 2, 0.5), ((20, 15, 11), 5, 10.0), ((70, 9, 8), 4, 2.0)]


@pytest.mark.parametrize("dims,R,mu", CASES)
def test_hessian_solve_matches_explicit_solve(dims, R, mu):
    dgn = _dgn()
    p = cpgen.small_problem(500 + R, dims, R, c=0.4)
    A = p.init
    rng = np.random.default_rng(9 + R)
    V = [rng.standard_normal((I, R)) for I in dims]
    J = brute.jacobian(A)
    H = J.T @ J + mu * np.eye(J.shape[1])
    want = np.linalg.solve(H, brute.param_vec(V))
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        print(f"hessian_solve dims={dims} R={R} mu={mu}", flush=True)
        X = ctx.hessian_solve(dims, R, dgn.to_device_factors(A), dgn.to_device_factors(V), mu)
        got = brute.param_vec(dgn.to_host_factors(X))
        assert _rel(got, want) < 1e-9, _rel(got, want)
        # H X = V through the block-form product (no H formed)
        HX = brute.hessian_matvec(A, dgn.to_host_factors(X))
        res = brute.param_vec(HX) + mu * got - brute.param_vec(V)
        assert np.linalg.norm(res) < 1e-9 * np.linalg.norm(brute.param_vec(V))
    finally:
        ctx.close()


def test_hessian_solve_of_the_gradient_is_the_step():
    # dgn_step is the solve with V = the gradient: same da to rounding
    dgn = _dgn()
    dims, R, mu = (30, 25, 20), 4, 3.0
    p = cpgen.small_problem(61, dims, R)
    Y = cp.as_tensor(p.y, dims)
    G = cp.fast_step(Y, p.init, mu).g
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        A = dgn.to_device_factors(p.init)
        out, _ = ctx.dgn_step(torch.from_numpy(p.y).cuda(), dims, R, A, mu)
        da = np.concatenate([(o - a).ravel() for o, a in zip(dgn.to_host_factors(out), p.init)])
        X = ctx.hessian_solve(dims, R, A, dgn.to_device_factors(G), mu)
        got = np.concatenate([x.ravel() for x in dgn.to_host_factors(X)])
        assert _rel(got, da) < 1e-10
    finally:
        ctx.close()


def test_hessian_solve_with_the_iterative_solver():
    dgn = _dgn()
    dims, R, mu = (40, 30, 20), 6, 1.0
    p = cpgen.small_problem(62, dims, R)
    rng = np.random.default_rng(3)
    V = [rng.standard_normal((I, R)) for I in dims]
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        A = dgn.to_device_factors(p.init)
        Xd = ctx.hessian_solve(dims, R, A, dgn.to_device_factors(V), mu)
        Xc = ctx.hessian_solve(dims, R, A, dgn.to_device_factors(V), mu,
                               dgn.opts(solver=1, cg_max_iters=500, cg_tol=1e-12))
        from test_gpu_cg import cond_S
        kappa = cond_S(p.init, mu)
        a = np.concatenate([x.ravel() for x in dgn.to_host_factors(Xc)])
        b = np.concatenate([x.ravel() for x in dgn.to_host_factors(Xd)])
        assert _rel(a, b) <= 10 * kappa * 1e-12 + 1e-11
    finally:
        ctx.close()


def test_hessian_solve_rejects_bad_arguments():
    dgn = _dgn()
    dims, R = (6, 5, 4), 2
    p = cpgen.small_problem(63, dims, R)
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        A = dgn.to_device_factors(p.init)
        V = dgn.to_device_factors([np.ones((I, R)) for I in dims])
        for mu in (0.0, -1.0, float("nan")):
            with pytest.raises(dgn.DgnError) as e:
                ctx.hessian_solve(dims, R, A, V, mu)
            assert e.value.status == -1
        with pytest.raises(dgn.DgnError) as e:
            ctx.hessian_solve((6, 5), R, A[:2], V[:2], 1.0)
        assert e.value.status == -1
    finally:
        ctx.close()


@pytest.mark.parametrize("dims,R,mu", [((9, 8, 7), 3, 1.0), ((7, 6, 5, 4), 2, 0.5)])
def test_hessian_solve_complex_matches_explicit_solve(dims, R, mu):
    # Section 5: (J^H J + mu I)^-1 v with the complex Jacobian of Lemma B.1
    dgn = _dgn()
    p = cpgen.small_problem(520 + R, dims, R, c=0.4, complex_=True)
    A = p.init
    rng = np.random.default_rng(19 + R)
    V = [rng.standard_normal((I, R)) + 1j * rng.standard_normal((I, R)) for I in dims]
    J = brute.jacobian(A)
    H = J.conj().T @ J + mu * np.eye(J.shape[1])
    want = np.linalg.solve(H, brute.param_vec(V))
    ctx = dgn.Context(0, dgn.workspace_size(dims, R, torch.complex128) + (16 << 20))
    try:
        print(f"hessian_solve complex dims={dims} R={R} mu={mu}", flush=True)
        X = ctx.hessian_solve(dims, R, dgn.to_device_factors(A), dgn.to_device_factors(V), mu)
        got = brute.param_vec(dgn.to_host_factors(X))
        assert _rel(got, want) < 1e-9, _rel(got, want)
    finally:
        ctx.close()
