"""Status paths of the boundary, the damping rules of Section 4.5, and the CG
attempt counters, through the C ABI.

* A non-finite tensor entry reaches the error and the step: DGN_ENONFINITE
  from dgn_step and cp_fit (and a failing server request is retired with that
  status while the others finish with the results they have alone).
* A damped Gram (Gamma^(n) + mu I) that is singular to working precision:
  DGN_ESINGULAR from dgn_step; inside a fit the trial is rejected instead.  Built exactly: two equal columns in every factor with
  squared norm 2 make Gamma^(n) = 4 * ones(2, 2); mu = 1e-300 vanishes in
  4 + mu, and the second Cholesky pivot is 4 - 2 * 2 = 0 in floating point.
* A zero column: H + mu I stays positive definite, so the step is defined and
  equals the explicit-Jacobian solve; the ALS update (mu = 0) is singular.
* mu > 1e30 stops the fit (Section 4.5).  From mu0 = 1e29 the step is below
  the rounding of the factors (|da| ~ |g| / mu), the candidate equals the
  factors, every trial is rejected, and mu grows 1e29 -> 2e29 -> 4e29 ->
  8e29 -> 1.6e30 (four trials) under the printed doubling and 1e29 -> 2e29
  -> 8e29 -> 6.4e30 (three) under Nielsen's rule.
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


def _nan_problem(dtype=torch.float64):
    p = cpgen.small_problem(9, (12, 10, 8), 3, c=0.3, snr_db=30.0)
    y = p.y.copy()
    y[37] = np.nan
    return p, torch.from_numpy(y).to(dtype).cuda()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_nan_tensor_step_nonfinite(ctx, dtype):
    dgn = _dgn()
    p, y = _nan_problem(dtype)
    with pytest.raises(dgn.DgnError) as e:
        ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(p.init), 1.0)
    assert e.value.status == -4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_nan_tensor_fit_nonfinite(ctx, dtype):
    dgn = _dgn()
    p, y = _nan_problem(dtype)
    with pytest.raises(dgn.DgnError) as e:
        ctx.cp_fit(y, p.dims, p.R, dgn.to_device_factors(p.init), 1.0, 0.0, 5)
    assert e.value.status == -4


def _equal_column_factors(dims):
    A = []
    for I in dims:
        v = np.zeros(I)
        v[0] = v[1] = 1.0  # squared norm 2
        A.append(np.asfortranarray(np.stack([v, v], axis=1)))
    return A


def test_singular_damped_gram_step(ctx):
    dgn = _dgn()
    dims = (4, 3, 5)
    A = _equal_column_factors(dims)
    y = np.random.default_rng(3).standard_normal(int(np.prod(dims)))
    with pytest.raises(dgn.DgnError) as e:
        ctx.dgn_step(torch.from_numpy(y).cuda(), dims, 2, dgn.to_device_factors(A), 1e-300)
    assert e.value.status == -3


def test_zero_column_step_defined_als_singular(ctx):
    dgn = _dgn()
    p = cpgen.small_problem(4, (6, 5, 4), 3, c=0.2, snr_db=30.0)
    A0 = [a.copy() for a in p.init]
    A0[1][:, 2] = 0.0
    y = torch.from_numpy(p.y).cuda()
    out, info = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(A0), 0.5)
    bda, _, _ = brute.plain_step(p.y, A0, 0.5)
    da = [g - a for g, a in zip(dgn.to_host_factors(out), A0)]
    assert _rel(cp.flat(da), cp.flat(bda)) < 1e-9
    with pytest.raises(dgn.DgnError) as e:
        ctx.cp_als(y, p.dims, p.R, dgn.to_device_factors(A0), 1)
    assert e.value.status == -3


@pytest.mark.parametrize("case", ["zero_first_block", "zero_second_block", "equal_columns"])
def test_semidefinite_gram_step(ctx, case):
    """C_n singular at R = 20 (two 16-column blocks in the factorisation of C_n):
    a zero column in either block, or two equal columns of one factor (the
    pivot falls to rounding level in the second block).  H + mu I stays
    positive definite, and the step equals the explicit-Jacobian solve."""
    dgn = _dgn()
    p = cpgen.small_problem(9, (14, 13, 12), 20, c=0.3, snr_db=30.0)
    A0 = [a.copy() for a in p.init]
    if case == "zero_first_block":
        A0[1][:, 2] = 0.0
    elif case == "zero_second_block":
        A0[0][:, 18] = 0.0
    else:
        A0[2][:, 17] = A0[2][:, 5]
    print(f"semidefinite C_n step case={case}", flush=True)
    y = torch.from_numpy(p.y).cuda()
    out, info = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(A0), 0.5)
    bda, _, _ = brute.plain_step(p.y, A0, 0.5)
    da = [g - a for g, a in zip(dgn.to_host_factors(out), A0)]
    err = _rel(cp.flat(da), cp.flat(bda))
    print(f"  rel err vs explicit solve {err:.2e}", flush=True)
    assert err < 1e-9


@pytest.mark.parametrize("batched", [False, True])
def test_singular_trials_rejected_in_fit(ctx, batched):
    """In a fit, a trial whose damped Gram is singular in FP64 is rejected and mu
    doubles; the fit goes on and returns no error.  The equal-column factors of
    the step test with mu0 = 1e-17: 4 + mu rounds to 4 for mu = 1e-17, 2e-17 and
    4e-17 (half an ulp of 4 is 4.4e-16), so all three trials are singular."""
    dgn = _dgn()
    dims = (4, 3, 5)
    A = _equal_column_factors(dims)
    y = torch.from_numpy(np.random.default_rng(3).standard_normal(int(np.prod(dims)))).cuda()
    Ad = dgn.to_device_factors(A)
    if batched:
        fi = ctx.cp_fit_batched([(y, dims, 2, Ad, 1e-17)], 0.0, 3)[0]
    else:
        fi = ctx.cp_fit(y, dims, 2, Ad, 1e-17, 0.0, 3)
    assert fi["iters"] == 3 and fi["accepted"] == 0 and fi["reason"] == dgn.STOP_MAX_IT
    assert fi["mu"] == 8e-17
    got = dgn.to_host_factors(Ad)
    assert all(np.array_equal(g, a) for g, a in zip(got, A))


@pytest.mark.parametrize("rule,trials", [(0, 4), (1, 3)])
def test_mu_overflow_stop(ctx, rule, trials):
    dgn = _dgn()
    p = cpgen.small_problem(6, (10, 9, 8), 3, c=0.4, snr_db=30.0)
    Y = cp.as_tensor(p.y, p.dims)
    A = dgn.to_device_factors(p.init)
    fi = ctx.cp_fit(torch.from_numpy(p.y).cuda(), p.dims, p.R, A, 1e29, 0.0, 50, dgn.opts(mu_rule=rule))
    fr = cp.fit(Y, p.init, mu0=1e29, tol=0.0, max_iters=50, mu_rule=("paper", "nielsen")[rule])
    assert fr["reason"] == cp.STOP_MU and fr["iters"] == trials and fr["accepted"] == 0
    assert fi["reason"] == dgn.STOP_MU and fi["iters"] == trials and fi["accepted"] == 0
    assert abs(fi["mu"] - fr["mu"]) <= 1e-12 * fr["mu"]


def _reject_heavy():
    # strongly collinear: a run of rejected trials early on.  At mu0 = 0.1 the
    # trajectory is well posed: the oracle's fLMa and fLMb (two rounding orders)
    # agree on mu to 1.3e-11 over 25 trials (at mu0 = 1e-6 the step's scaling
    # null-space components, amplified by 1/mu, reach the gain ratio)
    return cpgen.small_problem(14, (20, 15, 10), 3, c=0.95, snr_db=30.0)


def test_mu_rule_nielsen_matches_oracle(ctx):
    dgn = _dgn()
    p = _reject_heavy()
    Y = cp.as_tensor(p.y, p.dims)
    y = torch.from_numpy(p.y).cuda()
    for k in (3, 10, 25):
        A = dgn.to_device_factors(p.init)
        fi = ctx.cp_fit(y, p.dims, p.R, A, 0.1, 0.0, k, dgn.opts(mu_rule=dgn.MU_NIELSEN))
        fr = cp.fit(Y, p.init, mu0=0.1, tol=0.0, max_iters=k, mu_rule="nielsen", trace=True)
        rejected = sum(not h["accepted"] for h in fr["hist"])
        print(f"  {k} trials: accepted {fi['accepted']}/{fr['accepted']}, rejected (oracle) {rejected}, "
              f"mu {fi['mu']:.6e}/{fr['mu']:.6e}", flush=True)
        assert fi["iters"] == fr["iters"] and fi["accepted"] == fr["accepted"]
        assert abs(fi["mu"] - fr["mu"]) <= 1e-9 * fr["mu"]
        got = dgn.to_host_factors(A)
        diff = brute.jacobian_matvec(fr["A"], [g - r for g, r in zip(got, fr["A"])])
        assert np.linalg.norm(diff) <= 1e-9 * np.linalg.norm(cp.full(fr["A"]))
    # the two rules part ways on this problem (a long run of rejections)
    A = dgn.to_device_factors(p.init)
    fp = ctx.cp_fit(y, p.dims, p.R, A, 0.1, 0.0, 25)
    fq = cp.fit(Y, p.init, mu0=0.1, tol=0.0, max_iters=25, mu_rule="paper")
    assert fp["accepted"] == fq["accepted"] and abs(fp["mu"] - fq["mu"]) <= 1e-9 * fq["mu"]
    assert fq["accepted"] != fr["accepted"]


def test_batched_mu_rule_nielsen_matches_cp_fit(ctx):
    dgn = _dgn()
    # problems with early runs of rejections whose trajectories are well posed at these mu0
    # (the oracle's fLMa and fLMb agree on mu to <= 6e-11)
    specs = [(14, (20, 15, 10), 3, 0.95, 0.1), (15, (12, 12, 12), 6, 0.7, 1.0), (13, (16, 14, 12), 5, 0.8, 1.0)]
    ps = [cpgen.small_problem(s, d, R, c=c, snr_db=30.0) for s, d, R, c, _ in specs]
    mu0s = [m for *_, m in specs]
    o = dgn.opts(mu_rule=dgn.MU_NIELSEN)
    facs = [dgn.to_device_factors(p.init) for p in ps]
    ys = [torch.from_numpy(p.y).cuda() for p in ps]
    infos = ctx.cp_fit_batched([(ys[b], p.dims, p.R, facs[b], mu0s[b]) for b, p in enumerate(ps)], 0.0, 12, o)
    for b, p in enumerate(ps):
        A = dgn.to_device_factors(p.init)
        fi = ctx.cp_fit(ys[b], p.dims, p.R, A, mu0s[b], 0.0, 12, o)
        fr = cp.fit(cp.as_tensor(p.y, p.dims), p.init, mu0=mu0s[b], tol=0.0, max_iters=12, mu_rule="nielsen",
                    trace=True)
        assert any(not h["accepted"] for h in fr["hist"])
        assert infos[b]["accepted"] == fi["accepted"] == fr["accepted"]
        assert abs(infos[b]["mu"] - fr["mu"]) <= 1e-9 * fr["mu"]
        assert abs(fi["mu"] - fr["mu"]) <= 1e-9 * fr["mu"]


def test_bad_mu_rule_rejected(ctx):
    dgn = _dgn()
    p = cpgen.small_problem(1, (4, 4, 4), 2)
    with pytest.raises(dgn.DgnError) as e:
        ctx.cp_fit(torch.from_numpy(p.y).cuda(), p.dims, p.R, dgn.to_device_factors(p.init), 1.0, 0.0, 2,
                   dgn.opts(mu_rule=7))
    assert e.value.status == -1


@pytest.mark.parametrize("serve_batch", [0, 1])
def test_server_retires_failing_request(serve_batch):
    """A request with a NaN entry is retired with DGN_ENONFINITE while the others
    finish with the results they have alone (through the slots, or with the
    batch lane on, the order-3 ones and the failing one through the lane)."""
    dgn = _dgn()
    specs = [((20, 18, 16), 3, 21), ((16, 14, 12, 6), 4, 22), ((24, 20, 10), 5, 23)]
    probs = [cpgen.small_problem(s, d, R, c=0.5, snr_db=25.0) for d, R, s in specs]
    ctx = dgn.Context(0, 1 << 28)
    alone = []
    for p in probs:
        A = dgn.to_device_factors(p.init)
        y = torch.from_numpy(p.y).cuda()
        if serve_batch and len(p.dims) == 3:
            info = ctx.cp_fit_batched([(y, p.dims, p.R, A, -1.0)], 1e-8, 30,
                                      dgn.opts(batched_launch=dgn.BATCH_PERSISTENT))[0]
        else:
            info = ctx.cp_fit(y, p.dims, p.R, A, -1.0, 1e-8, 30)
        info.pop("t_done")
        alone.append((dgn.to_host_factors(A), info))
    ctx.close()
    bad, ybad = _nan_problem()
    srv = dgn.Server(0, budget_bytes=64 << 20, max_slots=2, options=dgn.opts(serve_batch=serve_batch))
    keep = {}
    for k, p in enumerate(probs):
        A = dgn.to_device_factors(p.init)
        keep[k] = A
        srv.submit(torch.from_numpy(p.y).cuda(), p.dims, p.R, A, -1.0, 1e-8, 30, tag=k)
        if k == 0:
            srv.submit(ybad, bad.dims, bad.R, dgn.to_device_factors(bad.init), -1.0, 1e-8, 30, tag=99)
    srv.wait_idle()
    res = {r["tag"]: r for r in srv.poll()}
    srv.close()
    assert set(res) == {0, 1, 2, 99}
    assert res[99]["status"] == -4
    assert res[99]["lane"] == serve_batch
    for k in range(3):
        assert res[k]["status"] == 0
        assert res[k]["lane"] == int(serve_batch and len(probs[k].dims) == 3)
        info = dict(res[k]["info"])
        info.pop("t_done")
        assert info == alone[k][1]
        for a, b in zip(dgn.to_host_factors(keep[k]), alone[k][0]):
            assert np.array_equal(a, b)


def test_cg_attempt_counters(ctx):
    """DGN_SOLVER_AUTO: a well-conditioned system converges within the cap and
    reports the same count as a converged and as an attempted solve; at the true
    factors of a collinear tensor with widely spread component norms and a small
    mu the attempt is abandoned at a checkpoint (every 10 iterations from the
    20th), below the cap, and the step equals the direct one."""
    dgn = _dgn()
    p = cpgen.cfg3(seed=8, dims=(40, 36, 30), R=12)
    y = torch.from_numpy(p.y).cuda()
    mu0 = cp.mu0_from_tau(p.init, 1e-3)
    o = dgn.opts(solver=1, cg_max_iters=100)
    out, info = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(p.init), mu0, o)
    print(f"  random start: cg_iters {info['cg_iters']} attempt {info['cg_attempt_iters']}", flush=True)
    assert 0 < info["cg_iters"] <= 100 and info["cg_attempt_iters"] == info["cg_iters"]
    mu = 1e-2 * cp.mu0_from_tau(p.truth, 1e-3)
    out, info = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(p.truth), mu, o)
    ref, rinfo = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(p.truth), mu)
    print(f"  true factors: cg_iters {info['cg_iters']} attempt {info['cg_attempt_iters']}", flush=True)
    assert info["cg_iters"] == -1 and rinfo["cg_iters"] == -1 and rinfo["cg_attempt_iters"] == -1
    assert 20 <= info["cg_attempt_iters"] < 100 and info["cg_attempt_iters"] % 10 == 0
    for a, b in zip(dgn.to_host_factors(out), dgn.to_host_factors(ref)):
        assert np.array_equal(a, b)
