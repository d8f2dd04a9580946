"""Parity of the mixed-precision path and of the shapes at the edge of the
library's limits, through the C ABI, against the FP64 oracle.

Bars (derived from the arithmetic; measured values are printed):
* BF16 tensor, MTTKRP against the MTTKRP of the BF16-rounded tensor in FP64:
  the factors enter the BF16 matrix cores as hi + lo pairs, each rounded to
  nearest, so a factor entry is carried to 2^-18 relative (2^-17 for the
  product of two); products and partial sums are FP32 (2^-24 per operation
  over a few hundred terms, random-walk growth) and the slab partials are
  reduced in FP64.  Normwise bar 4e-5.  Without the lo half a factor entry
  keeps only 2^-9 and the error is ~1e-3, 25x the bar.
* FP32 tensor, one step in the residual form (E = Y - Y_hat formed in FP32,
  MTTKRP of E): each entry of E is off by at most a few u32 (|y| + |y_hat|)
  (u32 = 2^-24), so by Cauchy-Schwarz the gradient block n is off by at most
  3 u32 ||(|Y| + |Y_hat|)_(n)|| ||KR_n|| (KR_n the Khatri-Rao product of the
  other factors), and the damped solve, ||(H + mu I)^-1|| <= 1/mu, passes
  that on to the step.  The test computes this first-order bound per case
  (1e-3 .. 4e-2 of ||da|| here; the errors are independent, so the measured
  ones sit two orders lower); a wrong sign or a dropped term in E is O(1).
* Fits: once the fit has switched to the residual form its error is
  sum(E^2) with E in FP32, so eps is resolved to about u32 = 6e-8; fits that
  converge to the same minimum therefore agree on the final eps to 1e-6
  (the target for the mixed path), the FP64 fit to 1e-9.
* Direct step at ranks above 32 (up to the library's limit of 64): the same
  1e-9 bar as at small ranks, against the plain explicit-Jacobian solve (the
  definition of the step) on tensors small enough to form J.
"""
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


def _q(y, dtype):
    """The tensor rounded to `dtype` on the device and the same values in FP64 for the oracle."""
    t = torch.from_numpy(y).to(dtype)
    return t, t.to(torch.float64).numpy()


BF16_SHAPES = [((20, 20, 20), 3), ((70, 65, 3), 4), ((130, 9, 5, 4), 5), ((64, 64, 64), 8),
               ((33, 200, 2), 30), ((17, 19, 4, 3), 64), ((90, 70, 60), 16)]


@pytest.mark.parametrize("shape", BF16_SHAPES)
def test_mttkrp_bf16_split_factors(ctx, shape):
    dims, R = shape
    print(f"bf16 mttkrp dims={dims} R={R}", flush=True)
    p = cpgen.small_problem(11 * len(dims) + R, dims, R, c=0.3, snr_db=20.0)
    yq, yref = _q(p.y, torch.bfloat16)
    Y = cp.as_tensor(yref, dims)
    dgn = _dgn()
    M, _ = ctx.dgn_mttkrp(yq.cuda(), dims, R, dgn.to_device_factors(p.init))
    got = dgn.to_host_factors(M)
    errs = [_rel(got[n], cp.mttkrp(Y, p.init, n)) for n in range(len(dims))]
    print("  rel errs", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) < 4e-5, errs


RESID_SHAPES = [((20, 20, 20), 3), ((70, 9, 65), 5), ((12, 11, 10, 9), 6), ((40, 30, 20), 10),
                ((66, 130, 70), 8)]


@pytest.mark.parametrize("shape", RESID_SHAPES)
def test_step_fp32_residual_pass_matches_oracle(ctx, shape):
    """dgn_step on an FP32 tensor with the residual-corrected pass (resid_switch < 0)
    against the oracle's step on the same FP32-rounded values."""
    dims, R = shape
    print(f"fp32 residual step dims={dims} R={R}", flush=True)
    p = cpgen.small_problem(5 * len(dims) + R, dims, R, c=0.5, snr_db=25.0)
    yq, yref = _q(p.y, torch.float32)
    Y = cp.as_tensor(yref, dims)
    dgn = _dgn()
    mu = 1.0
    out, info = ctx.dgn_step(yq.cuda(), dims, R, dgn.to_device_factors(p.init), mu,
                             dgn.opts(resid_switch=-1.0))
    got = dgn.to_host_factors(out)
    ref = cp.fast_step(Y, p.init, mu)
    da = [g - a for g, a in zip(got, p.init)]
    err = _rel(cp.flat(da), cp.flat(ref.dA))
    ny2 = float(np.sum(Y ** 2))
    e_old = cp.residual_norm2(Y, p.init)
    e_new = cp.residual_norm2(Y, ref.A_new)
    u32 = 2.0 ** -24
    absE = np.abs(Y) + np.abs(cp.full(p.init))
    bound = 3 * u32 * sum(np.linalg.norm(cp.unfold(absE, n)) * np.linalg.norm(cp.kr_except(p.init, n))
                          for n in range(len(dims))) / mu / np.linalg.norm(cp.flat(ref.dA))
    print(f"  step rel err {err:.2e} (bound {bound:.2e}), err2_old rel {abs(info['err2_old'] - e_old) / ny2:.2e}, "
          f"err2_new rel {abs(info['err2_new'] - e_new) / ny2:.2e}", flush=True)
    assert err < bound
    # sum(E^2) with E in FP32: each entry off by ~u32 (|y| + |y_hat|)
    assert abs(info["err2_old"] - e_old) <= 1e-6 * (ny2 + e_old)
    assert abs(info["err2_new"] - e_new) <= 1e-6 * (ny2 + e_new)


def _fit_problem():
    # converges from a random start to the 30 dB noise floor well inside 80 trials
    return cpgen.small_problem(41, (60, 50, 40), 4, c=0.5, snr_db=30.0)


@pytest.fixture(scope="module")
def oracle_fits():
    """Oracle fits of the same problem on the FP64 values and on the FP32-rounded values."""
    p = _fit_problem()
    out = {}
    for name, dtype in (("f64", torch.float64), ("f32", torch.float32)):
        _, yref = _q(p.y, dtype)
        out[name] = cp.fit(cp.as_tensor(yref, p.dims), p.init, mu0=-1.0, tol=0.0, max_iters=80)
    return p, out


@pytest.mark.parametrize("path", ["f64", "f32", "f32+bf16"])
def test_fit_mixed_precision_matches_oracle(ctx, oracle_fits, path):
    """cp_fit from an FP32 tensor (and an FP32 tensor with a BF16 copy for the plain
    passes) reaches the oracle's final eps on the FP32-rounded tensor to 1e-6, after
    switching to the residual-corrected pass; the FP64 path to 1e-9."""
    p, fr = oracle_fits
    dgn = _dgn()
    ref = fr["f64" if path == "f64" else "f32"]
    dtype = torch.float64 if path == "f64" else torch.float32
    yq, _ = _q(p.y, dtype)
    yq = yq.cuda()
    o = dgn.opts(y_bf16=yq.to(torch.bfloat16)) if path == "f32+bf16" else dgn.opts()
    A = dgn.to_device_factors(p.init)
    fi = ctx.cp_fit(yq, p.dims, p.R, A, -1.0, 0.0, 80, o)
    d = abs(fi["eps"] - ref["eps"])
    got = dgn.to_host_factors(A)
    mdiff = _rel(cp.full(got).ravel(), cp.full(ref["A"]).ravel())
    print(f"  {path}: eps {fi['eps']:.10f} oracle {ref['eps']:.10f} |d| {d:.2e} "
          f"resid_iters {fi['resid_iters']} accepted {fi['accepted']}/{ref['accepted']} "
          f"model diff {mdiff:.2e}", flush=True)
    assert fi["iters"] == 80
    assert ref["eps"] < 0.05  # converged to the noise floor (30 dB: 0.0316)
    if path == "f64":
        assert d < 1e-9
        assert mdiff < 1e-8
    else:
        assert fi["resid_iters"] > 0
        assert d < 1e-6
        assert mdiff < 1e-5


HIGH_RANK = [((14, 12, 10), 33), ((12, 11, 10), 40), ((10, 9, 8), 48), ((7, 6, 5), 64), ((5, 4, 3, 3), 36)]


@pytest.mark.parametrize("mu", [1.0, 30.0])
@pytest.mark.parametrize("shape", HIGH_RANK)
def test_step_high_rank_matches_explicit_solve(ctx, shape, mu):
    """Ranks 33..64 (sub-blocks, SYRK and Cholesky tiles of the largest size)
    against the plain damped Gauss-Newton step with J formed explicitly."""
    dims, R = shape
    print(f"high-rank step dims={dims} R={R} mu={mu}", flush=True)
    p = cpgen.small_problem(3 * len(dims) + R, dims, R, c=0.3, snr_db=25.0)
    dgn = _dgn()
    out, info = ctx.dgn_step(torch.from_numpy(p.y).cuda(), dims, R, dgn.to_device_factors(p.init), mu)
    got = dgn.to_host_factors(out)
    bda, g, _ = brute.plain_step(p.y, p.init, mu)
    da = [x - a for x, a in zip(got, p.init)]
    err = _rel(cp.flat(da), cp.flat(bda))
    print(f"  rel err vs explicit solve {err:.2e}", flush=True)
    assert err < 1e-9
    if R <= 40:
        ref = cp.fast_step(cp.as_tensor(p.y, dims), p.init, mu)
        assert _rel(cp.flat(da), cp.flat(ref.dA)) < 1e-9


COMPLEX_HIGH = [((26, 24, 22), 24), ((8, 7, 6), 32), ((34, 33, 32), 32)]


@pytest.mark.parametrize("mu", [1.0, 30.0])
@pytest.mark.parametrize("shape", COMPLEX_HIGH)
def test_step_complex_high_rank(ctx, shape, mu):
    """Complex ranks 24 and 32 (the limit) against the oracle's fast step and,
    where J is small enough, the explicit (J^H J + mu I)^-1 J^H e solve."""
    dims, R = shape
    print(f"complex high-rank step dims={dims} R={R} mu={mu}", flush=True)
    p = cpgen.small_problem(17 * len(dims) + R, dims, R, c=0.4, snr_db=25.0, complex_=True)
    dgn = _dgn()
    out, info = ctx.dgn_step(torch.from_numpy(p.y).cuda(), dims, R, dgn.to_device_factors(p.init), mu)
    got = dgn.to_host_factors(out)
    da = [x - a for x, a in zip(got, p.init)]
    ref = cp.fast_step(cp.as_tensor(p.y, dims), p.init, mu)
    err = _rel(cp.flat(da), cp.flat(ref.dA))
    print(f"  rel err vs oracle {err:.2e}", flush=True)
    assert err < 1e-9
    if R * sum(dims) <= 1500:
        bda, _, _ = brute.plain_step(p.y, p.init, mu)
        assert _rel(cp.flat(da), cp.flat(bda)) < 1e-9


@pytest.fixture(scope="module")
def cfg2_problem():
    p = cpgen.cfg2()
    mu = cp.mu0_from_tau(p.init, 1e-3)
    ref = cp.fast_step(cp.as_tensor(p.y, p.dims), p.init, mu)
    return p, mu, ref


def test_cfg2_first_step_fp64(ctx, cfg2_problem):
    """100^4, R = 10 (correlation 0.95, 20 dB): the first step from the FP64 tensor
    at full size against the oracle, to the FP64 bar."""
    p, mu, ref = cfg2_problem
    dgn = _dgn()
    y = torch.from_numpy(p.y).cuda()
    out, info = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(p.init), mu)
    got = dgn.to_host_factors(out)
    da = [x - a for x, a in zip(got, p.init)]
    err = _rel(cp.flat(da), cp.flat(ref.dA))
    print(f"  cfg2 fp64 step rel err {err:.2e} (mu {mu:.3e})", flush=True)
    assert np.linalg.norm(cp.flat(ref.g)) / np.linalg.norm(cp.flat(ref.M)) > 1e-5
    assert err < 1e-9
    del y
    torch.cuda.empty_cache()


def test_cfg2_first_step_fp32(ctx, cfg2_problem):
    """The same step from the FP32 tensor (plain FP32 MFMA pass): the oracle's step on
    the FP64 values, to the FP32 gradient's accuracy (MTTKRP ~2e-7 relative, carried
    through the damped solve): bar 1e-4."""
    p, mu, ref = cfg2_problem
    dgn = _dgn()
    y = torch.from_numpy(p.y).to(torch.float32).cuda()
    out, info = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(p.init), mu)
    got = dgn.to_host_factors(out)
    da = [x - a for x, a in zip(got, p.init)]
    err = _rel(cp.flat(da), cp.flat(ref.dA))
    print(f"  cfg2 fp32 step rel err {err:.2e}", flush=True)
    assert err < 1e-4
    del y
    torch.cuda.empty_cache()
