"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances (derived from the arithmetic, stated per test):
* FP64 tensor pass: normwise relative error <= 1e-12 (J-term sums in FP64).
* FP32 pass: <= 2e-5 (FP32 products of FP32-rounded factors, FP32 partial
  sums over at most a few hundred slabs, FP64 final reduction).
* BF16 tensor: <= 4e-5 against the MTTKRP of the BF16-rounded tensor (the
  factors enter the BF16 matrix cores as hi + lo pairs, 2^-18 relative each;
  FP32 products and partial sums).
* FP64 step: relative update error <= 1e-9 on unconverged inputs
  (||g|| / ||M|| >= 1e-5), the bar of the stated target.
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


MTTKRP_SHAPES = [
    ((20, 20, 20), 3), ((70, 65, 3), 4), ((130, 9, 5, 4), 5), ((5, 6, 7, 3, 2), 2),
    ((64, 64, 64), 8), ((1, 40, 3), 2), ((3, 1, 150), 1), ((33, 200, 2), 30), ((17, 19, 4, 3), 64),
]


def _quantize(y, dtype):
    t = torch.from_numpy(y).to(dtype)
    return t, t.to(torch.float64).numpy()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5),
                                       (torch.bfloat16, 4e-5)])
@pytest.mark.parametrize("shape", MTTKRP_SHAPES)
def test_mttkrp_all_modes(ctx, shape, dtype, tol):
    dims, R = shape
    print(f"mttkrp dims={dims} R={R} dtype={dtype}", flush=True)
    p = cpgen.small_problem(len(dims) * 100 + R, dims, R, c=0.3, snr_db=20.0)
    yq, yref = _quantize(p.y, dtype)
    Y = cp.as_tensor(yref, dims)
    dgn = _dgn()
    M, inner = ctx.dgn_mttkrp(yq.cuda(), dims, R, dgn.to_device_factors(p.init))
    got = dgn.to_host_factors(M)
    for n in range(len(dims)):
        ref = cp.mttkrp(Y, p.init, n)
        assert _rel(got[n], ref) < tol, (n, _rel(got[n], ref))
    ref_inner = float(np.sum(Y * cp.full(p.init)))
    assert abs(inner - ref_inner) <= tol * np.linalg.norm(yref) * np.linalg.norm(cp.full(p.init))


STEP_SHAPES = [((4, 3, 5), 1), ((5, 4, 3), 2), ((4, 4, 4, 3), 3), ((3, 3, 3, 3, 3), 2),
               ((20, 20, 20), 3), ((70, 9, 65), 5), ((12, 11, 10, 9), 6), ((40, 30, 20), 10)]


@pytest.mark.parametrize("mu", [1e-2, 1.0, 30.0])
@pytest.mark.parametrize("shape", STEP_SHAPES)
def test_step_fp64_matches_oracle(ctx, shape, mu):
    dims, R = shape
    print(f"step dims={dims} R={R} mu={mu}", flush=True)
    p = cpgen.small_problem(7 * len(dims) + R, dims, R, c=0.5, snr_db=25.0)
    Y = cp.as_tensor(p.y, dims)
    dgn = _dgn()
    out, info = ctx.dgn_step(torch.from_numpy(p.y).cuda(), dims, R, dgn.to_device_factors(p.init), mu)
    got = dgn.to_host_factors(out)
    ref = cp.fast_step(Y, p.init, mu)
    assert np.linalg.norm(cp.flat(ref.g)) / np.linalg.norm(cp.flat(ref.M)) > 1e-5
    da = [g - a for g, a in zip(got, p.init)]
    assert _rel(cp.flat(da), cp.flat(ref.dA)) < 1e-9
    e_old = cp.residual_norm2(Y, p.init)
    e_new = cp.residual_norm2(Y, ref.A_new)
    # residuals: FP64 sums; the new one also carries the step's own 1e-9-level difference
    assert abs(info["err2_old"] - e_old) <= 1e-12 * np.sum(Y ** 2)
    assert abs(info["err2_new"] - e_new) <= 1e-10 * (np.sum(Y ** 2) + e_new)
    assert abs(info["denom"] - cp.gain_denominator(ref.dA, ref.g, mu)) <= 1e-9 * abs(info["denom"])
    if np.prod(dims) <= 200:
        bda, _, _ = brute.plain_step(p.y, p.init, mu)
        assert _rel(cp.flat(da), cp.flat(bda)) < 1e-9


# ranks at the edges of the 16-column blocks of the R x R factorisations (R
# padded to 16 ceil(R / 16) with the identity: one block with and without
# padding, two blocks with 15 and with 0 padding rows)
EDGE_RANKS = [((17, 16, 15), 15), ((18, 17, 16), 16), ((19, 18, 17), 17), ((16, 15, 14), 31),
              ((15, 14, 13), 32)]


@pytest.mark.parametrize("mu", [1e-2, 30.0])
@pytest.mark.parametrize("shape", EDGE_RANKS)
def test_step_block_edge_ranks_match_oracle(ctx, shape, mu):
    dims, R = shape
    print(f"edge-rank step dims={dims} R={R} mu={mu}", flush=True)
    p = cpgen.small_problem(5 * R + 1, dims, R, c=0.5, snr_db=25.0)
    dgn = _dgn()
    out, info = ctx.dgn_step(torch.from_numpy(p.y).cuda(), dims, R, dgn.to_device_factors(p.init), mu)
    got = dgn.to_host_factors(out)
    ref = cp.fast_step(cp.as_tensor(p.y, dims), p.init, mu)
    da = [g - a for g, a in zip(got, p.init)]
    err = _rel(cp.flat(da), cp.flat(ref.dA))
    print(f"  rel err vs oracle {err:.2e}", flush=True)
    assert err < 1e-9
    assert abs(info["denom"] - cp.gain_denominator(ref.dA, ref.g, mu)) <= 1e-9 * abs(info["denom"])


def test_step_zero_gradient_exact_rank(ctx):
    dims, R = (9, 8, 7), 3
    p = cpgen.small_problem(3, dims, R, c=0.4, snr_db=None)
    dgn = _dgn()
    y = cpgen.cp_tensor(p.init)
    out, info = ctx.dgn_step(torch.from_numpy(y).cuda(), dims, R, dgn.to_device_factors(p.init), 0.1)
    got = dgn.to_host_factors(out)
    assert np.linalg.norm(cp.flat(got) - cp.flat(p.init)) < 1e-10 * np.linalg.norm(cp.flat(p.init))
    assert info["err2_old"] < 1e-20 * np.sum(y ** 2)


def test_fit_cfg1_matches_oracle(ctx):
    """20^3, R=3, mode-1 correlation 0.9, 30 dB, mu0 = 1, 50 trials (first workload)."""
    p = cpgen.cfg1()
    Y = cp.as_tensor(p.y, p.dims)
    dgn = _dgn()
    y = torch.from_numpy(p.y).cuda()
    # early trials: factors agree to the step bar
    for k in (1, 4, 8):
        A = dgn.to_device_factors(p.init)
        fi = ctx.cp_fit(y, p.dims, p.R, A, p.mu0, 0.0, k)
        fr = cp.fit(Y, p.init, mu0=p.mu0, tol=0.0, max_iters=k)
        got = dgn.to_host_factors(A)
        diff = brute.jacobian_matvec(fr["A"], [g - r for g, r in zip(got, fr["A"])])
        assert np.linalg.norm(diff) <= 1e-9 * np.linalg.norm(cp.full(fr["A"]))
        assert fi["iters"] == fr["iters"] and fi["accepted"] == fr["accepted"]
        assert abs(fi["mu"] - fr["mu"]) <= 1e-9 * fr["mu"]
    A = dgn.to_device_factors(p.init)
    fi = ctx.cp_fit(y, p.dims, p.R, A, p.mu0, p.tol, p.max_iters)
    fr = cp.fit(Y, p.init, mu0=p.mu0, tol=p.tol, max_iters=p.max_iters)
    assert fi["iters"] == 50 and fi["reason"] == dgn.STOP_MAX_IT
    assert abs(fi["eps"] - fr["eps"]) < 1e-6
    assert abs(fi["eps"] - np.sqrt(cp.residual_norm2(Y, dgn.to_host_factors(A)) / np.sum(Y ** 2))) < 1e-12


@pytest.mark.parametrize("normalize", [0, 1, 2])
def test_fit_normalisations(ctx, normalize):
    p = cpgen.small_problem(5, (15, 12, 10, 8), 4, c=0.6, snr_db=30.0)
    Y = cp.as_tensor(p.y, p.dims)
    dgn = _dgn()
    A = dgn.to_device_factors(p.init)
    fi = ctx.cp_fit(torch.from_numpy(p.y).cuda(), p.dims, p.R, A, 0.5, 0.0, 6,
                    dgn.opts(normalize=normalize))
    fr = cp.fit(Y, p.init, mu0=0.5, tol=0.0, max_iters=6,
                normalize={0: "balanced", 1: "unit", 2: "none"}[normalize])
    got = dgn.to_host_factors(A)
    assert _rel(cp.flat(got), cp.flat(fr["A"])) < 1e-9
    assert fi["accepted"] == fr["accepted"]


def test_fit_noiseless_recovery(ctx):
    dims, R = (10, 9, 8), 3
    p = cpgen.small_problem(21, dims, R, c=0.6, snr_db=None)
    rng = np.random.default_rng(1)
    A0 = [a + 1e-2 * rng.standard_normal(a.shape) for a in p.truth]
    dgn = _dgn()
    A = dgn.to_device_factors(A0)
    fi = ctx.cp_fit(torch.from_numpy(p.y).cuda(), dims, R, A, -1.0, 0.0, 60)
    assert fi["eps"] <= 1e-12


def test_tau_mu0_rule(ctx):
    p = cpgen.small_problem(2, (8, 7, 6), 2, c=0.2, snr_db=30.0)
    dgn = _dgn()
    A = dgn.to_device_factors(p.init)
    fi = ctx.cp_fit(torch.from_numpy(p.y).cuda(), p.dims, p.R, A, -1.0, 0.0, 0, dgn.opts(tau=1e-2))
    assert abs(fi["mu0"] - cp.mu0_from_tau(p.init, 1e-2)) <= 1e-12 * fi["mu0"]
    assert fi["iters"] == 0


def test_invalid_arguments(ctx):
    dgn = _dgn()
    p = cpgen.small_problem(1, (4, 4, 4), 2)
    y = torch.from_numpy(p.y).cuda()
    A = dgn.to_device_factors(p.init)
    with pytest.raises(dgn.DgnError) as e:
        ctx.dgn_step(y, p.dims, p.R, A, 0.0)
    assert e.value.status == -1
    with pytest.raises(dgn.DgnError):
        ctx.cp_fit(y, p.dims, p.R, A, 1.0, -1.0, 3)
    small = dgn.Context(0, 4096)
    with pytest.raises(dgn.DgnError) as e:
        small.dgn_step(y, p.dims, p.R, A, 1.0)
    assert e.value.status == -2
    small.close()
