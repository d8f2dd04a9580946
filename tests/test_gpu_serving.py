"""Serving (dgn_server_*): admission by memory budget, concurrent slots, the
batch lane for requests within the batched shapes, and results identical alone
and in the mix (all kernels are deterministic, so the bar is bit-for-bit
equality of factors and fit info): a slot's result equals cp_fit's, a lane
result equals cp_fit_batched's for that fit alone."""
import numpy as np
import pytest
import torch

import cpgen

pytestmark = pytest.mark.gpu


def _dgn():
    from paper_1205_2584_amd import dgn
    return dgn


def _requests():
    specs = [((24, 20, 18), 4, torch.float64), ((16, 30, 22, 12), 5, torch.float32),
             ((40, 33, 28), 10, torch.float32), ((17, 19, 16), 18, torch.float64),
             ((50, 20, 12, 9), 3, torch.float32), ((64, 48, 40), 6, torch.float32),
             ((14, 12, 10), 5, torch.complex128), ((20, 18, 9, 6), 4, torch.complex64)]
    out = []
    for k, (dims, R, dt) in enumerate(specs):
        p = cpgen.small_problem(300 + k, dims, R, c=0.5, snr_db=20.0, complex_=dt.is_complex)
        out.append((p, dt))
    return out


def _lane_eligible(p, dt):
    return len(p.dims) == 3 and max(p.dims) <= 64 and p.R <= 8 and dt in (torch.float32, torch.float64)


def _alone(ctx, p, dt, tol, max_iters, lane):
    """The request run by itself: cp_fit, or (lane) cp_fit_batched on a batch of one."""
    dgn = _dgn()
    y = torch.from_numpy(p.y).to(dt).cuda()
    A = dgn.to_device_factors(p.init)
    if lane:
        info = ctx.cp_fit_batched([(y, p.dims, p.R, A, -1.0)], tol, max_iters,
                                  dgn.opts(batched_launch=dgn.BATCH_PERSISTENT))[0]
    else:
        info = ctx.cp_fit(y, p.dims, p.R, A, -1.0, tol, max_iters)
    return dgn.to_host_factors(A), info


def _same_info(a, b):
    # the in-batch completion time is a clock reading, not a result
    return {k: v for k, v in a.items() if k != "t_done"} == {k: v for k, v in b.items() if k != "t_done"}


@pytest.mark.parametrize("serve_batch", [0, 1])
def test_results_same_alone_and_in_mix(serve_batch):
    dgn = _dgn()
    reqs = _requests()
    ctx = dgn.Context(0, 1 << 30)
    alone = [_alone(ctx, p, dt, 1e-8, 40, serve_batch and _lane_eligible(p, dt)) for p, dt in reqs]
    ctx.close()
    assert sum(_lane_eligible(p, dt) for p, dt in reqs) == 2
    sizes = [dgn.workspace_size(p.dims, p.R, dt) for p, dt in reqs]
    srv = dgn.Server(0, budget_bytes=2 * max(sizes) + (4 << 20), max_slots=3,
                     options=dgn.opts(serve_batch=serve_batch))
    keep = []
    for k, (p, dt) in enumerate(reqs):
        y = torch.from_numpy(p.y).to(dt).cuda()
        A = dgn.to_device_factors(p.init)
        keep.append(A)
        srv.submit(y, p.dims, p.R, A, -1.0, 1e-8, 40, tag=k)
    srv.wait_idle()
    res = srv.poll()
    srv.close()
    assert len(res) == len(reqs)
    for r in res:
        k = r["tag"]
        assert r["status"] == 0
        assert r["lane"] == int(bool(serve_batch) and _lane_eligible(*reqs[k]))
        assert _same_info(r["info"], alone[k][1])
        got = dgn.to_host_factors(keep[k])
        for a, b in zip(got, alone[k][0]):
            assert np.array_equal(a, b)
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_batch_lane_groups_pending_requests():
    """Forty small requests (two stop settings) and two large ones submitted at
    once: the small ones run in the lane in batches of more than one, each
    grouped by (tol, max_iters), every result equal to its fit run alone."""
    dgn = _dgn()
    rng = np.random.default_rng(41)
    small = []
    for k in range(40):
        dims = tuple(int(v) for v in rng.integers(8, 65, size=3))
        R = int(rng.integers(2, 9))
        dt = torch.float32 if k % 3 else torch.float64
        small.append((cpgen.small_problem(500 + k, dims, R, c=float(rng.uniform(0, 0.9)), snr_db=25.0), dt,
                      1e-8, 30 if k % 2 else 45))
    large = [(cpgen.small_problem(600 + k, dims, R, c=0.5, snr_db=20.0), torch.float32, 1e-8, 30)
             for k, (dims, R) in enumerate([((80, 60, 50), 6), ((40, 30, 20, 10), 4)])]
    reqs = small + large
    ctx = dgn.Context(0, 1 << 30)
    alone = [_alone(ctx, p, dt, tol, it, k < len(small)) for k, (p, dt, tol, it) in enumerate(reqs)]
    ctx.close()
    srv = dgn.Server(0, budget_bytes=1 << 30, max_slots=2)
    keep = []
    for k, (p, dt, tol, it) in enumerate(reqs):
        y = torch.from_numpy(p.y).to(dt).cuda()
        A = dgn.to_device_factors(p.init)
        keep.append((y, A))
        srv.submit(y, p.dims, p.R, A, -1.0, tol, it, tag=k)
    srv.wait_idle()
    res = srv.poll(max_results=64)
    srv.close()
    assert len(res) == len(reqs)
    assert max(r["batch_size"] for r in res if r["lane"] == 1) > 1
    for r in res:
        k = r["tag"]
        assert r["status"] == 0
        assert r["lane"] == int(k < len(small))
        assert _same_info(r["info"], alone[k][1])
        for a, b in zip(dgn.to_host_factors(keep[k][1]), alone[k][0]):
            assert np.array_equal(a, b)
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_admission_respects_budget_and_rejects_oversize():
    dgn = _dgn()
    p = cpgen.small_problem(1, (40, 40, 40), 8)
    need = dgn.workspace_size(p.dims, p.R, torch.float64)
    srv = dgn.Server(0, budget_bytes=need + (1 << 20) + 4096, max_slots=4, options=dgn.opts(serve_batch=0))
    ys, fs = [], []
    for k in range(4):
        y = torch.from_numpy(p.y).cuda()
        A = dgn.to_device_factors(p.init)
        ys.append(y)
        fs.append(A)
        srv.submit(y, p.dims, p.R, A, -1.0, 0.0, 5, tag=k)
    peak = 0
    while True:
        used, running, queued = srv.stats()
        peak = max(peak, running)
        if running == 0 and queued == 0:
            break
    srv.wait_idle()
    res = srv.poll()
    assert len(res) == 4 and all(r["status"] == 0 for r in res)
    assert peak <= 1  # only one request fits the budget at a time
    # admitted in arrival order
    admits = sorted((r["t_admit"], r["tag"]) for r in res)
    assert [t for _, t in admits] == [0, 1, 2, 3]
    big = cpgen.small_problem(2, (64, 64, 64), 30)
    with pytest.raises(dgn.DgnError) as e:
        srv.submit(torch.from_numpy(big.y).cuda(), big.dims, big.R, dgn.to_device_factors(big.init))
    assert e.value.status == -6
    srv.close()
