"""Batched small fits (cp_fit_batched) against cp_fit and the FP64 oracle.

FP64 tensors run the residual form from the first trial in both paths, so
the same trials are accepted and the factors agree to the step bar
(<= 1e-9 relative, model space) on unconverged trials; final relative errors
agree to 1e-6 (the stated final-fit tolerance).  Graph replay and one-by-one
launches run identical kernels and must agree bit for bit.
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


def _problems(count, seed=4, dtype=torch.float64, max_dim=64):
    ps = cpgen.cfg4(seed=seed, count=count)
    out = []
    for p in ps:
        dims = tuple(min(d, max_dim) for d in p.dims)
        if dims != p.dims:
            q = cpgen.small_problem(p.meta["index"] + 1000 * seed, dims, p.R, c=p.meta["c"],
                                    snr_db=p.meta["snr_db"])
            p = q
        out.append(p)
    return out


def _same(a, b):
    """Fit infos equal in every field but the batch latency t_done (a clock reading)."""
    return {k: v for k, v in a.items() if k != "t_done"} == {k: v for k, v in b.items() if k != "t_done"}


def _run_batched(ctx, ps, dtype, tol, iters, **kw):
    dgn = _dgn()
    facs = [dgn.to_device_factors(p.init) for p in ps]
    ys = [torch.from_numpy(p.y).to(dtype).cuda() for p in ps]
    probs = [(ys[b], p.dims, p.R, facs[b], -1.0) for b, p in enumerate(ps)]
    infos = ctx.cp_fit_batched(probs, tol, iters, dgn.opts(**kw))
    return [dgn.to_host_factors(f) for f in facs], infos


def test_batched_matches_single_fits(ctx):
    dgn = _dgn()
    ps = _problems(12)
    for iters in (3, 30):
        facs, infos = _run_batched(ctx, ps, torch.float64, 0.0, iters)
        for b, p in enumerate(ps):
            print(f"fit {b} dims={p.dims} R={p.R} iters={iters}", flush=True)
            A = dgn.to_device_factors(p.init)
            fi = ctx.cp_fit(torch.from_numpy(p.y).cuda(), p.dims, p.R, A, -1.0, 0.0, iters)
            got = dgn.to_host_factors(A)
            assert infos[b]["iters"] == fi["iters"]
            assert abs(infos[b]["eps"] - fi["eps"]) < 1e-6
            if iters == 3:
                assert infos[b]["accepted"] == fi["accepted"]
                diff = brute.jacobian_matvec(got, [x - y for x, y in zip(facs[b], got)])
                assert np.linalg.norm(diff) <= 1e-9 * np.linalg.norm(cp.full(got))


def test_batched_matches_oracle(ctx):
    ps = _problems(4, seed=9)
    facs, infos = _run_batched(ctx, ps, torch.float64, 1e-8, 40)
    for b, p in enumerate(ps):
        Y = cp.as_tensor(p.y, p.dims)
        fr = cp.fit(Y, p.init, mu0=-1.0, tol=1e-8, max_iters=40)
        assert abs(infos[b]["eps"] - fr["eps"]) < 1e-6
        eps_direct = np.sqrt(cp.residual_norm2(Y, facs[b]) / np.sum(Y ** 2))
        assert abs(eps_direct - infos[b]["eps"]) < 1e-12


def test_batched_graph_replay_equals_eager(ctx):
    ps = _problems(10, seed=5)
    f1, i1 = _run_batched(ctx, ps, torch.float32, 1e-8, 24, graph=1, poll_every=8, batched_launch=1)
    f2, i2 = _run_batched(ctx, ps, torch.float32, 1e-8, 24, graph=0, poll_every=8, batched_launch=1)
    f3, i3 = _run_batched(ctx, ps, torch.float32, 1e-8, 24, graph=1, poll_every=3, batched_launch=1)
    for b in range(len(ps)):
        assert _same(i1[b], i2[b]) and _same(i1[b], i3[b])
        for x, y, z in zip(f1[b], f2[b], f3[b]):
            assert np.array_equal(x, y) and np.array_equal(x, z)


def test_batched_fp32_tensor_agrees(ctx):
    """FP32 data: the batch accumulates in FP64, cp_fit in FP32 MFMA; final fits agree to 1e-5."""
    dgn = _dgn()
    ps = _problems(6, seed=7)
    facs, infos = _run_batched(ctx, ps, torch.float32, 1e-9, 60)
    for b, p in enumerate(ps):
        A = dgn.to_device_factors(p.init)
        fi = ctx.cp_fit(torch.from_numpy(p.y).float().cuda(), p.dims, p.R, A, -1.0, 1e-9, 60)
        assert abs(infos[b]["eps"] - fi["eps"]) < 1e-5


def test_batched_rejects_unsupported(ctx):
    dgn = _dgn()
    p = cpgen.small_problem(1, (70, 8, 8), 3)
    with pytest.raises(dgn.DgnError) as e:
        _run_batched(ctx, [p], torch.float64, 0.0, 2)
    assert e.value.status == -1


def test_batched_persistent_equals_graph(ctx):
    """The persistent queue runs each fit with the same trial code as the per-trial
    launches: results are bit-identical, whatever the order the queue hands out."""
    dgn = _dgn()
    ps = _problems(40, seed=11)
    for dt in (torch.float32, torch.float64):
        f1, i1 = _run_batched(ctx, ps, dt, 1e-8, 60, batched_launch=1)
        assert ctx.batched_last_launch() == 1
        f2, i2 = _run_batched(ctx, ps, dt, 1e-8, 60, batched_launch=2)
        assert ctx.batched_last_launch() == 2
        for b in range(len(ps)):
            assert _same(i1[b], i2[b])
            for x, y in zip(f1[b], f2[b]):
                assert np.array_equal(x, y)


def test_batched_tuner_table(ctx):
    """AUTO: the first batch with a new (largest mode size, largest rank) key is timed
    in both shapes; the table records both figures and the faster shape, which the
    call then used (same results as that shape run explicitly)."""
    dgn = _dgn()
    ps = [cpgen.small_problem(900 + k, (40 + k, 33, 47 - k), 7, c=0.4, snr_db=30.0) for k in range(12)]
    f0, i0 = _run_batched(ctx, ps, torch.float32, 1e-8, 30)
    used = ctx.batched_last_launch()
    table = dgn.batched_tuning()
    print("tuning table", table, flush=True)
    imax = max(max(p.dims) for p in ps)
    ent = [e for e in table if e["imax_bucket"] == 16 * ((imax + 15) // 16) and e["rmax"] == max(p.R for p in ps)]
    assert len(ent) == 1
    e = ent[0]
    assert e["us_per_trial_graph"] > 0 and e["us_per_trial_persistent"] > 0
    assert e["launch"] == (2 if e["us_per_trial_persistent"] < e["us_per_trial_graph"] else 1)
    assert used == e["launch"]
    f1, i1 = _run_batched(ctx, ps, torch.float32, 1e-8, 30, batched_launch=used)
    for b in range(len(ps)):
        assert _same(i0[b], i1[b])
        for x, y in zip(f0[b], f1[b]):
            assert np.array_equal(x, y)


def test_batched_latency_recorded(ctx):
    """t_done: each fit's stop time within the batch, from the device clock."""
    ps = _problems(20, seed=13)
    for launch in (1, 2):
        _, infos = _run_batched(ctx, ps, torch.float32, 1e-8, 40, batched_launch=launch)
        t = [i["t_done"] for i in infos]
        assert all(x >= 0.0 for x in t) and max(t) > 0.0 and max(t) < 60.0
