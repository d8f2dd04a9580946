"""Complex tensors (Section 5) through the C ABI against the FP64 oracle.

MTTKRP with conjugated factors, the fast step (pinned by the explicit
(J^H J + mu I)^-1 J^H e solve on small shapes), and fits that follow the
oracle's trajectory."""
import numpy as np
import pytest
import torch

import cpgen
from oracle import brute, cp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1205_2584_amd import dgn
    c = dgn.Context(0, 1 << 30)
    yield c
    c.close()


def _dgn():
    from paper_1205_2584_amd import dgn
    return dgn


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


MTTKRP_SHAPES = [((20, 20, 20), 3), ((70, 45, 3), 4), ((33, 9, 5, 4), 5), ((5, 6, 7, 3, 2), 2),
                 ((64, 65, 31), 8), ((1, 40, 3), 2), ((40, 33, 9), 32), ((17, 19, 4, 3), 20)]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("shape", MTTKRP_SHAPES)
def test_mttkrp_complex(ctx, shape, dtype):
    dims, R = shape
    print(f"complex mttkrp dims={dims} R={R} dtype={dtype}", flush=True)
    p = cpgen.small_problem(len(dims) * 31 + R, dims, R, c=0.3, snr_db=20.0, complex_=True)
    yq = torch.from_numpy(p.y).to(dtype)
    yref = yq.to(torch.complex128).numpy()
    Y = cp.as_tensor(yref, dims)
    dgn = _dgn()
    M, inner = ctx.dgn_mttkrp(yq.cuda(), dims, R, dgn.to_device_factors(p.init))
    got = dgn.to_host_factors(M)
    for n in range(len(dims)):
        ref = cp.mttkrp(Y, p.init, n, conj=True)
        assert _rel(got[n], ref) < 1e-12, (n, _rel(got[n], ref))
    ref_inner = float(np.real(np.sum(Y * np.conj(cp.full(p.init)))))
    assert abs(inner - ref_inner) <= 1e-12 * np.linalg.norm(yref) * np.linalg.norm(cp.full(p.init))


STEP_SHAPES = [((4, 3, 5), 1), ((5, 4, 3), 2), ((4, 4, 4, 3), 3), ((3, 3, 3, 3, 3), 2),
               ((20, 20, 20), 3), ((40, 9, 35), 5), ((12, 11, 10, 9), 6), ((36, 30, 20), 10),
               ((24, 20, 18), 20)]


@pytest.mark.parametrize("mu", [1e-2, 1.0, 30.0])
@pytest.mark.parametrize("shape", STEP_SHAPES)
def test_step_complex_matches_oracle(ctx, shape, mu):
    dims, R = shape
    print(f"complex step dims={dims} R={R} mu={mu}", flush=True)
    p = cpgen.small_problem(13 * len(dims) + R, dims, R, c=0.5, snr_db=25.0, complex_=True)
    Y = cp.as_tensor(p.y, dims)
    dgn = _dgn()
    out, info = ctx.dgn_step(torch.from_numpy(p.y).cuda(), dims, R, dgn.to_device_factors(p.init), mu)
    got = dgn.to_host_factors(out)
    ref = cp.fast_step(Y, p.init, mu)
    assert np.linalg.norm(cp.flat(ref.g)) / np.linalg.norm(cp.flat(ref.M)) > 1e-5
    da = [g - a for g, a in zip(got, p.init)]
    assert _rel(cp.flat(da), cp.flat(ref.dA)) < 1e-9
    ny2 = float(np.sum(np.abs(Y) ** 2))
    e_old = cp.residual_norm2(Y, p.init)
    e_new = cp.residual_norm2(Y, ref.A_new)
    assert abs(info["err2_old"] - e_old) <= 1e-12 * ny2
    assert abs(info["err2_new"] - e_new) <= 1e-10 * (ny2 + e_new)
    assert abs(info["denom"] - cp.gain_denominator(ref.dA, ref.g, mu)) <= 1e-9 * abs(info["denom"])
    if np.prod(dims) <= 200:
        bda, _, _ = brute.plain_step(p.y, p.init, mu)
        assert _rel(cp.flat(da), cp.flat(bda)) < 1e-9


def test_step_complex_zero_gradient(ctx):
    dims, R = (9, 8, 7), 3
    p = cpgen.small_problem(3, dims, R, c=0.4, snr_db=None, complex_=True)
    dgn = _dgn()
    y = cpgen.cp_tensor(p.init)
    out, info = ctx.dgn_step(torch.from_numpy(y).cuda(), dims, R, dgn.to_device_factors(p.init), 0.1)
    got = dgn.to_host_factors(out)
    assert np.linalg.norm(cp.flat(got) - cp.flat(p.init)) < 1e-10 * np.linalg.norm(cp.flat(p.init))
    assert info["err2_old"] < 1e-20 * np.sum(np.abs(y) ** 2)


@pytest.mark.parametrize("shape", [((12, 10, 9), 3), ((8, 7, 6, 5), 4), ((30, 25, 20), 8)])
def test_fit_complex_matches_oracle(ctx, shape):
    dims, R = shape
    p = cpgen.small_problem(77 + R, dims, R, c=0.6, snr_db=25.0, complex_=True)
    Y = cp.as_tensor(p.y, dims)
    dgn = _dgn()
    y = torch.from_numpy(p.y).cuda()
    for k in (1, 3, 6):
        A = dgn.to_device_factors(p.init)
        fi = ctx.cp_fit(y, dims, R, A, -1.0, 0.0, k)
        fr = cp.fit(Y, p.init, mu0=-1.0, tol=0.0, max_iters=k)
        got = dgn.to_host_factors(A)
        diff = brute.jacobian_matvec(fr["A"], [g - r for g, r in zip(got, fr["A"])])
        assert np.linalg.norm(diff) <= 1e-9 * np.linalg.norm(cp.full(fr["A"]))
        assert fi["iters"] == fr["iters"] and fi["accepted"] == fr["accepted"]
        assert abs(fi["mu"] - fr["mu"]) <= 1e-9 * fr["mu"]
        assert abs(fi["eps"] - fr["eps"]) <= 1e-10


def test_fit_complex_noiseless_recovery(ctx):
    dims, R = (10, 9, 8), 3
    p = cpgen.small_problem(21, dims, R, c=0.6, snr_db=None, complex_=True)
    rng = np.random.default_rng(1)
    A0 = [a + 1e-2 * (rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)) for a in p.truth]
    dgn = _dgn()
    A = dgn.to_device_factors(A0)
    fi = ctx.cp_fit(torch.from_numpy(p.y).cuda(), dims, R, A, -1.0, 0.0, 60)
    assert fi["eps"] <= 1e-12


def test_complex_rank_limit(ctx):
    dgn = _dgn()
    p = cpgen.small_problem(4, (6, 5, 4), 2, complex_=True)
    with pytest.raises(dgn.DgnError):
        ctx.dgn_mttkrp(torch.from_numpy(p.y).cuda(), (6, 5, 4), 33,
                       [torch.zeros(33, I, dtype=torch.complex128, device="cuda") for I in (6, 5, 4)])
