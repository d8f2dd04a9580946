"""The iterative NR^2 solve (DGN_SOLVER_AUTO: conjugate gradients on the
structured SPD system S = I + W^T K W of Section 4.3, the direct Cholesky as
fallback) against the direct solve and the oracle.

Tolerance: CG stops at ||r|| <= cg_tol ||z||, so the solution y of S y = z is
within cond(S) cg_tol relative of the exact one.  The step da is a fixed linear
map of y plus terms that do not depend on it, so the tests allow
10 cond(S) cg_tol ||da|| on top of the direct step's own rounding (1e-11 relative),
with cond(S) computed in NumPy from the same factors: S depends only on the
Grams C_n and on mu (its spectrum does not depend on the choice of square-root
factors in W).  When CG does not converge, or for shapes it does not take
(N > 4 or R > 32), the step must be bit-identical to the direct one.
"""
import numpy as np
import pytest
import torch

import cpgen
from oracle import cp

pytestmark = pytest.mark.gpu


def _dgn():
    from paper_1205_2584_amd import dgn
    return dgn


def cond_S(A, mu):
    """cond(S), S = I + W^T K W, W = blkdiag(X_n (x) L_n), X X^T = (Gamma_n + mu I)^-1, L L^T = C_n."""
    C = cp.grams(A)
    G = cp.gammas(C)
    R = A[0].shape[1]
    R2 = R * R
    N = len(A)
    W = np.zeros((N * R2, N * R2))
    for n in range(N):
        X = np.linalg.cholesky(np.linalg.inv(G[n] + mu * np.eye(R)))
        L = np.linalg.cholesky(C[n])
        W[n * R2:(n + 1) * R2, n * R2:(n + 1) * R2] = np.kron(X, L)
    S = np.eye(N * R2) + W.T @ cp.kernel_K(C) @ W
    ev = np.linalg.eigvalsh((S + S.T) / 2)
    return float(ev[-1] / ev[0])


def _rel(a, b):
    return float(np.linalg.norm(np.concatenate([x.ravel() for x in a]) - np.concatenate([x.ravel() for x in b]))
                 / np.linalg.norm(np.concatenate([x.ravel() for x in b])))


CASES = [
    ((40, 30, 20), 5, 1.0),
    ((33, 28, 45), 12, 10.0),
    ((20, 18, 25, 9), 6, 1.0),
    ((36, 34, 32), 32, 100.0),   # the largest rank CG takes
    ((70, 65, 60), 30, 1.0),
]


@pytest.mark.parametrize("dims,R,mu", CASES)
def test_cg_step_matches_direct_and_oracle(dims, R, mu):
    dgn = _dgn()
    p = cpgen.small_problem(300 + R, dims, R, c=0.5, snr_db=30.0)
    Y = cp.as_tensor(p.y, dims)
    y = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        print(f"cg step dims={dims} R={R} mu={mu}", flush=True)
        A = dgn.to_device_factors(p.init)
        out_d, info_d = ctx.dgn_step(y, dims, R, A, mu)
        out_c, info_c = ctx.dgn_step(y, dims, R, A, mu, dgn.opts(solver=1, cg_max_iters=500, cg_tol=1e-12))
        assert info_d["cg_iters"] == -1
        assert 0 < info_c["cg_iters"] <= 500, info_c["cg_iters"]
        kappa = cond_S(p.init, mu)
        tol = 10 * kappa * 1e-12 + 1e-11
        dd = [o - a for o, a in zip(dgn.to_host_factors(out_d), p.init)]
        dc = [o - a for o, a in zip(dgn.to_host_factors(out_c), p.init)]
        assert _rel(dc, dd) <= tol, (_rel(dc, dd), tol, kappa)
        ref = cp.fast_step(Y, p.init, mu)
        da_ref = [a1 - a0 for a1, a0 in zip(ref.A_new, p.init)]
        assert _rel(dc, da_ref) <= tol + 1e-9
    finally:
        ctx.close()


def test_cg_fallback_is_the_direct_step():
    # one CG iteration cannot reach the tolerance: the direct solve runs and the
    # step is bit-identical to the direct one
    dgn = _dgn()
    dims, R, mu = (40, 30, 20), 6, 1.0
    p = cpgen.small_problem(41, dims, R)
    y = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        A = dgn.to_device_factors(p.init)
        out_d, _ = ctx.dgn_step(y, dims, R, A, mu)
        out_c, info = ctx.dgn_step(y, dims, R, A, mu, dgn.opts(solver=1, cg_max_iters=1))
        assert info["cg_iters"] == -1
        for a, b in zip(out_c, out_d):
            assert torch.equal(a, b)
    finally:
        ctx.close()


@pytest.mark.parametrize("dims,R", [((20, 18, 16), 40), ((9, 8, 7, 6, 5), 3)])
def test_cg_unsupported_shapes_use_the_direct_solve(dims, R):
    dgn = _dgn()
    p = cpgen.small_problem(43, dims, R)
    y = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        A = dgn.to_device_factors(p.init)
        out_d, _ = ctx.dgn_step(y, dims, R, A, 1.0)
        out_c, info = ctx.dgn_step(y, dims, R, A, 1.0, dgn.opts(solver=1))
        assert info["cg_iters"] == -1
        for a, b in zip(out_c, out_d):
            assert torch.equal(a, b)
    finally:
        ctx.close()


def test_cg_rejects_bad_options():
    dgn = _dgn()
    dims, R = (10, 11, 12), 3
    p = cpgen.small_problem(44, dims, R)
    y = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        A = dgn.to_device_factors(p.init)
        for kw in ({"solver": 2}, {"solver": 1, "cg_tol": 0.0}, {"solver": 1, "cg_max_iters": -1}):
            with pytest.raises(dgn.DgnError) as e:
                ctx.dgn_step(y, dims, R, A, 1.0, dgn.opts(**kw))
            assert e.value.status == -1
            with pytest.raises(dgn.DgnError) as e:
                ctx.cp_fit(y, dims, R, dgn.to_device_factors(p.init), 1.0, 0.0, 3, dgn.opts(**kw))
            assert e.value.status == -1
    finally:
        ctx.close()


def test_cg_fit_matches_direct_fit():
    dgn = _dgn()
    dims, R = (30, 28, 26), 4
    p = cpgen.small_problem(45, dims, R, c=0.6, snr_db=30.0)
    y = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size(dims, R) + (16 << 20))
    try:
        Ad = dgn.to_device_factors(p.init)
        info_d = ctx.cp_fit(y, dims, R, Ad, -1.0, 0.0, 30)
        Ac = dgn.to_device_factors(p.init)
        info_c = ctx.cp_fit(y, dims, R, Ac, -1.0, 0.0, 30, dgn.opts(solver=1, cg_max_iters=400, cg_tol=1e-13))
        assert info_d["cg_trials"] == 0
        assert info_c["cg_trials"] > 0 and info_c["cg_iters"] >= info_c["cg_trials"]
        assert info_c["iters"] == info_d["iters"] == 30
        # same trajectory within the solver tolerance: the final errors agree
        assert abs(info_c["eps"] - info_d["eps"]) <= 1e-6 * info_d["eps"]
        # a CG that never converges leaves every trial to the direct solve: bit-identical to the direct fit
        Ao = dgn.to_device_factors(p.init)
        info_o = ctx.cp_fit(y, dims, R, Ao, -1.0, 0.0, 30, dgn.opts(solver=1, cg_max_iters=1))
        assert info_o["cg_trials"] == 0
        for a, b in zip(Ao, Ad):
            assert torch.equal(a, b)
    finally:
        ctx.close()


def test_cg_step_full_size_500cube():
    """The 500^3 R=30 FP32 workload at its first trial (random factors, mu0 of
    the tau rule): the CG step agrees with the direct step within the bound."""
    dgn = _dgn()
    p = cpgen.cfg3(3)
    dims, R = p.dims, p.R
    y = torch.from_numpy(p.y.astype(np.float32)).cuda()
    mu = cp.mu0_from_tau(p.init, 1e-3)
    ctx = dgn.Context(0, dgn.workspace_size(dims, R, torch.float32) + (16 << 20))
    try:
        print("cg step 500^3 R=30", flush=True)
        A = dgn.to_device_factors(p.init)
        out_d, _ = ctx.dgn_step(y, dims, R, A, mu)
        out_c, info = ctx.dgn_step(y, dims, R, A, mu, dgn.opts(solver=1, cg_max_iters=500, cg_tol=1e-12))
        assert 0 < info["cg_iters"] <= 500
        kappa = cond_S(p.init, mu)
        dd = [o - a for o, a in zip(dgn.to_host_factors(out_d), p.init)]
        dc = [o - a for o, a in zip(dgn.to_host_factors(out_c), p.init)]
        assert _rel(dc, dd) <= 10 * kappa * 1e-12 + 1e-11, (_rel(dc, dd), kappa)
    finally:
        ctx.close()


# ---- complex tensors (Section 5): CG on the Hermitian system ---------------------


def cond_Phi(Y, A, mu):
    """cond(S) of the complex step from the eigenvalues of Phi_1 = I + Psi K,
    which has the spectrum of S = I + W^H K W (Psi = W W^H)."""
    ev = np.linalg.eigvals(cp.fast_step(Y, A, mu).Phi)
    ev = np.abs(ev)
    return float(ev.max() / ev.min())


@pytest.mark.parametrize("dims,R,mu", [((20, 18, 16), 4, 1.0), ((12, 10, 9, 8), 3, 1.0), ((36, 34, 32), 16, 10.0)])
def test_cg_complex_step_matches_direct(dims, R, mu):
    dgn = _dgn()
    p = cpgen.small_problem(700 + R, dims, R, c=0.4, snr_db=30.0, complex_=True)
    Y = cp.as_tensor(p.y, dims)
    y = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size(dims, R, torch.complex128) + (16 << 20))
    try:
        print(f"cg complex step dims={dims} R={R} mu={mu}", flush=True)
        A = dgn.to_device_factors(p.init)
        out_d, info_d = ctx.dgn_step(y, dims, R, A, mu)
        out_c, info_c = ctx.dgn_step(y, dims, R, A, mu, dgn.opts(solver=1, cg_max_iters=500, cg_tol=1e-12))
        assert info_d["cg_iters"] == -1
        assert 0 < info_c["cg_iters"] <= 500, info_c["cg_iters"]
        kappa = cond_Phi(Y, p.init, mu)
        dd = [o - a for o, a in zip(dgn.to_host_factors(out_d), p.init)]
        dc = [o - a for o, a in zip(dgn.to_host_factors(out_c), p.init)]
        assert _rel(dc, dd) <= 10 * kappa * 1e-12 + 1e-11, (_rel(dc, dd), kappa)
    finally:
        ctx.close()


def test_cg_complex_fallback_and_unsupported_rank_are_the_direct_step():
    dgn = _dgn()
    for dims, R, kw in (((20, 18, 16), 4, {"cg_max_iters": 1}), ((24, 22, 20), 17, {})):
        p = cpgen.small_problem(800 + R, dims, R, complex_=True)
        y = torch.from_numpy(p.y).cuda()
        ctx = dgn.Context(0, dgn.workspace_size(dims, R, torch.complex128) + (16 << 20))
        try:
            A = dgn.to_device_factors(p.init)
            out_d, _ = ctx.dgn_step(y, dims, R, A, 1.0)
            out_c, info = ctx.dgn_step(y, dims, R, A, 1.0, dgn.opts(solver=1, **kw))
            assert info["cg_iters"] == -1
            for a, b in zip(out_c, out_d):
                assert torch.equal(a, b)
        finally:
            ctx.close()
