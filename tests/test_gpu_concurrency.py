"""Fits running at the same time on one GPU, each on its own context and stream,
must give bit-for-bit the results they give alone.

Every kernel is deterministic, so any difference means that one launch depends on
the order in which its own workgroups are dispatched (for example a tile that one
workgroup overwrites while another of the same launch still has to read it), or
that two contexts share state. Other fits filling the compute units change that
dispatch order, which a fit alone on the GPU never shows. The problems use
R >= 9 so that the N R^2 system spans several 64-wide tiles and every phase of
the tiled Cholesky has panel and update workgroups side by side.

Other launches on the compute units also delay a wave's LDS stores relative to
the other waves of its workgroup, so a barrier reached with a store still in
flight gives wrong values only under load; the tensor-pass test below is sized
to reach the LDS flushes inside the pass's slab loop."""
import queue
import threading

import numpy as np
import pytest
import torch

import cpgen

pytestmark = pytest.mark.gpu


def _dgn():
    from paper_1205_2584_amd import dgn
    return dgn


def _pool():
    rng = np.random.default_rng(77)
    out = []
    for k in range(12):
        N = 3 + (k % 2)
        dims = tuple(int(rng.integers(16, 49)) for _ in range(N))
        R = int(rng.integers(9, 17)) if N == 3 else int(rng.integers(9, 12))
        out.append(cpgen.small_problem(7700 + k, dims, R, c=float(rng.uniform(0.3, 0.9)), snr_db=20.0))
    return out


def _fit(ctx, dgn, y, p, max_iters):
    A = dgn.to_device_factors(p.init)
    try:
        info = ctx.cp_fit(y, p.dims, p.R, A, -1.0, 1e-8, max_iters)
        status = 0
    except dgn.DgnError as e:
        info, status = None, e.status
    torch.cuda.current_stream().synchronize()
    return status, info, [a.cpu().numpy().copy() for a in A]


def test_concurrent_fits_match_sequential():
    dgn = _dgn()
    pool = _pool()
    ys = [torch.from_numpy(p.y.astype(np.float32)).cuda() for p in pool]
    max_iters = 60
    ctx = dgn.Context(0, 1 << 30)
    ref = [_fit(ctx, dgn, ys[k], p, max_iters) for k, p in enumerate(pool)]
    ctx.close()
    assert all(r[0] == 0 for r in ref)

    order = [k % len(pool) for k in range(4 * len(pool))]
    jobs = queue.Queue()
    for j, k in enumerate(order):
        jobs.put((j, k))
    out, errors = {}, []

    def worker():
        try:
            torch.cuda.set_device(0)
            s = torch.cuda.Stream()
            c = dgn.Context(0, 1 << 30)
            with torch.cuda.stream(s):
                while True:
                    try:
                        j, k = jobs.get_nowait()
                    except queue.Empty:
                        break
                    out[j] = _fit(c, dgn, ys[k], pool[k], max_iters)
            c.close()
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=worker) for _ in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    bad = []
    for j, k in enumerate(order):
        st, info, A = out[j]
        r = ref[k]
        same = st == r[0] and info == r[1] and all(np.array_equal(a, b) for a, b in zip(A, r[2]))
        if not same:
            bad.append((j, k, st, pool[k].dims, pool[k].R))
    assert not bad, bad


# A tensor whose 64 x 64 output tiles each walk far more than 16 slabs of the
# trailing index in one workgroup, so that the per-slab partials of the
# trailing modes are flushed from LDS inside the slab loop (every 16 slabs),
# not only after it: tiles 2 x 1, Q = 206 * 117 = 24102 slabs over 254 chunks,
# 95 slabs and 5 flushes inside the loop per workgroup.  A flush that reads
# LDS before another wave's last store has landed shows up as a few wrong
# entries of M_3 and M_4 (four consecutive ranks at one trailing index) in a
# few percent of the calls, and only while other launches share the compute
# units.
_PASS_DIMS = (117, 39, 206, 117)


@pytest.mark.parametrize("dtype,R", [(torch.float32, 16), (torch.float32, 40), (torch.bfloat16, 30)])
def test_concurrent_tensor_passes_bit_exact(dtype, R):
    dgn = _dgn()
    g = torch.Generator(device="cuda")
    g.manual_seed(4242 + R)
    J = int(np.prod(_PASS_DIMS))
    y = torch.randn(J, generator=g, device="cuda", dtype=torch.float32).to(dtype).contiguous()
    A = [torch.randn((R, I), generator=g, device="cuda", dtype=torch.float64) for I in _PASS_DIMS]
    torch.cuda.synchronize()
    ws = dgn.workspace_size(_PASS_DIMS, R, dtype) + (16 << 20)
    ctx = dgn.Context(0, ws)
    M, _ = ctx.dgn_mttkrp(y, _PASS_DIMS, R, A)
    ref = [m.cpu().numpy() for m in M]
    ctx.close()
    calls, errors, bad = 60, [], []

    def worker(k):
        try:
            torch.cuda.set_device(0)
            s = torch.cuda.Stream()
            c = dgn.Context(0, ws)
            with torch.cuda.stream(s):
                for i in range(calls):
                    M, _ = c.dgn_mttkrp(y, _PASS_DIMS, R, A)
                    for n, (a, b) in enumerate(zip([m.cpu().numpy() for m in M], ref)):
                        if not np.array_equal(a, b):
                            bad.append((k, i, n, int(np.count_nonzero(a != b))))
            s.synchronize()
            c.close()
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    assert not bad, bad[:10]
