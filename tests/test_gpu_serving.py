"""Serving (dgn_server_*): admission by memory budget, concurrent slots, and
results identical alone and in the mix (all kernels are deterministic, so the
bar is bit-for-bit equality of factors and fit info)."""
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


def test_results_same_alone_and_in_mix():
    dgn = _dgn()
    reqs = _requests()
    ctx = dgn.Context(0, 1 << 30)
    alone = []
    for p, dt in reqs:
        y = torch.from_numpy(p.y).to(dt).cuda()
        A = dgn.to_device_factors(p.init)
        info = ctx.cp_fit(y, p.dims, p.R, A, -1.0, 1e-8, 40)
        alone.append((dgn.to_host_factors(A), info))
    ctx.close()
    sizes = [dgn.workspace_size(p.dims, p.R, dt) for p, dt in reqs]
    srv = dgn.Server(0, budget_bytes=2 * max(sizes) + (4 << 20), max_slots=3)
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
        assert r["info"] == alone[k][1]
        got = dgn.to_host_factors(keep[k])
        for a, b in zip(got, alone[k][0]):
            assert np.array_equal(a, b)
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_admission_respects_budget_and_rejects_oversize():
    dgn = _dgn()
    p = cpgen.small_problem(1, (40, 40, 40), 8)
    need = dgn.workspace_size(p.dims, p.R, torch.float64)
    srv = dgn.Server(0, budget_bytes=need + (1 << 20) + 4096, max_slots=4)
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
