"""Benchmark: damped Gauss-Newton (fLM) iterations per second for a 3-way
500 x 500 x 500 dense tensor at rank R = 30 (NR^2 = 2700) on one MI355X.

A step is one trial of the fit (Algorithm 1 with the damping of Section 4.5):
Gram/Hadamard products, damped inverses, gradient rows, the NR^2 system
(assembly, Cholesky, solves), the factor update, the tensor pass at the
candidate (all-mode MTTKRP) and the damping control.  The tensor is stored in
FP32 (plus a BF16 copy); the MTTKRP accumulates in FP32; everything after it
is FP64.  Inputs are seeded and synthetic (truth with component norms 1..1e3,
correlation 0.9 in mode 3, 25 dB noise) and resident in HBM before timing.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]

Prints one JSON line.  The CPU baseline times the FP64 oracle on a bounded
sample (one trial of the same workload) on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def workload(name):
    import cpgen
    if name == "500cube_r30":
        return cpgen.cfg3()
    if name == "100pow4_r10":
        return cpgen.cfg2()
    if name == "20cube_r3":
        return cpgen.cfg1()
    raise SystemExit(f"unknown workload {name}")


def chol_flops(N, R):
    """FP64 flops of the factor_solve phase per trial: Cholesky of the
    (N-1)R^2 Schur complement (nt^3/3) plus its forward and backward
    substitutions (nt^2 each)."""
    nt = (N - 1) * R * R
    return nt ** 3 / 3.0 + 2.0 * nt * nt


def schur_update_flops(N, R):
    """FP64 flops of the Schur update S_tt - B B^T in the assemble phase: from the
    structure of B for R <= 32 (three R x R products per (a, a') and block pair),
    else the lower half of the dense nt x nt product with inner dimension R^2."""
    if R <= 32:
        return 6.0 * R ** 5 * (N - 1) * N / 2
    nt = (N - 1) * R * R
    return float(nt) * nt * R * R


# HBM bytes per unit of work, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs
# (scaled against a 1 GiB copy), for the 500^3 R=30 workload.  Each entry holds
# for the kernel source and compiler flags whose SHA-256 prefix is given; once
# either changes the figure no longer describes the kernel and is reported as
# null.
TRAFFIC = {
    "factor_solve": (("paper_1205_2584_amd/csrc/chol.hip", "paper_1205_2584_amd/csrc/panel.hpp"),
                     "2f62f32b09a52b6d", 827900571),
    "tensor_pass_f32": (("paper_1205_2584_amd/csrc/tensor_pass.hip",), "cec26df43e38f726", 517666929),
    "tensor_pass_bf16": (("paper_1205_2584_amd/csrc/tensor_pass.hip",), "cec26df43e38f726", 268064024),
}


def traffic(key, workload_name):
    if workload_name != "500cube_r30":
        return None
    paths, sha, nbytes = TRAFFIC[key]
    return nbytes if kernel_sha(paths) == sha else None


def kernel_sha(paths):
    """SHA-256 prefix of a kernel's sources together with the library's compiler flags."""
    import hashlib
    from paper_1205_2584_amd import build
    h = hashlib.sha256()
    for path in paths:
        with open(os.path.join(ROOT, path), "rb") as f:
            h.update(f.read())
    flags = [f for i, f in enumerate(build.FLAGS) if f != "-I" and not (i and build.FLAGS[i - 1] == "-I")]
    h.update(" ".join(flags).encode())  # include paths differ between machines
    return h.hexdigest()[:16]


def cpu_baseline(p, gpu_check, seconds_cap=30.0):
    """Times the FP64 oracle (fast step + direct residual) on a bounded sample of
    the same fit, and hands its first step (at the initial factors) to
    `gpu_check`, which compares the GPU's results at full size against it."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import cp
    Y = cp.as_tensor(p.y, p.dims)
    A = [np.array(a) for a in p.init]
    mu = cp.mu0_from_tau(A, 1e-3)
    t0 = time.perf_counter()
    n = 0
    first = None
    while True:
        st = cp.fast_step(Y, A, mu)
        cp.residual_norm2(Y, st.A_new)
        n += 1
        if first is None:
            first = st
        if time.perf_counter() - t0 > seconds_cap / 3 or n >= 3:
            break
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    base = {"value": n / dt, "unit": "iters/s", "cores": threads, "kind": "oracle",
            "nproc": len(os.sched_getaffinity(0)), "cpu_model": model,
            "sample": f"{n} trial step(s) (fast step + residual) of the same 500^3 R=30 fit, FP64 NumPy"}
    return base, gpu_check(first, mu)


def bench_batched(dgn, torch, count=1024, max_iters=200, tol=1e-8, seq_sample=128):
    """1024 independent 3-way fits (I_n ~ U{8..64}, R ~ U{2..8}), FP32 tensors, in
    one cp_fit_batched call: the launch shape the library's tuner picks (AUTO), and
    each shape forced; per-fit latency inside the batch from the device clock; the
    same fits one cp_fit at a time on a sample of `seq_sample` fits."""
    import numpy as np
    import cpgen
    ps = cpgen.cfg4(count=count, max_iters=max_iters, tol=tol)
    ys = [torch.from_numpy(p.y.astype(np.float32)).cuda() for p in ps]
    ctx = dgn.Context(0, 2 << 30)

    def run(launch):
        probs = [(ys[b], p.dims, p.R, dgn.to_device_factors(p.init), -1.0) for b, p in enumerate(ps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = ctx.cp_fit_batched(probs, tol, max_iters, dgn.opts(batched_launch=launch))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos, ctx.batched_last_launch()

    names = {1: "graph", 2: "persistent"}
    run(0)  # warm-up; the first AUTO call also times both shapes and records the choice
    dt, infos, used = run(0)
    shapes = {}
    for launch in (1, 2):
        d, _, _ = run(launch)
        shapes[names[launch]] = round(count / d, 1)
    trials = sum(i["iters"] for i in infos)
    lat = np.array([i["t_done"] for i in infos]) * 1e3
    # algorithmic work of the run: each trial of fit b takes one pass over its
    # FP32 tensor (J_b entries) with 4 J_b R_b FP64 flops (all-mode MTTKRP)
    Js = [int(np.prod(p.dims)) for p in ps]
    flops = sum(4.0 * J * p.R * i["iters"] for J, p, i in zip(Js, ps, infos))
    tbytes = sum(4.0 * J * i["iters"] for J, i in zip(Js, infos))
    tf = flops / dt / 1e12
    # sequential baseline on a sample
    t1 = time.perf_counter()
    for b in range(seq_sample):
        A = dgn.to_device_factors(ps[b].init)
        ctx.cp_fit(ys[b], ps[b].dims, ps[b].R, A, -1.0, tol, max_iters)
    torch.cuda.synchronize()
    dseq = time.perf_counter() - t1
    ctx.close()
    seq_rate = seq_sample / dseq
    imax = max(max(p.dims) for p in ps)
    rmax = max(p.R for p in ps)
    table = [e for e in dgn.batched_tuning() if e["imax_bucket"] == 16 * ((imax + 15) // 16) and e["rmax"] == rmax]
    return {"fits": count, "fits_per_s": round(count / dt, 1), "wall_s": round(dt, 3),
            "launch": names.get(used, used), "fits_per_s_by_launch": shapes,
            "tuner_entry": table[0] if table else None,
            "trials_total": trials, "mean_trials": round(trials / count, 1),
            "sequential_cp_fit_fits_per_s": round(seq_rate, 2),
            "sequential_sample": f"first {seq_sample} fits, one cp_fit call each",
            "speedup_vs_sequential": round((count / dt) / seq_rate, 1),
            "p50_latency_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_latency_ms": round(float(np.percentile(lat, 99)), 2),
            "latency_note": "per-fit time from the batch's first initial state to the fit's stop (device clock)",
            "roofline_batched": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None,
                                 "algorithmic_flops": flops, "tensor_GBs": round(tbytes / dt / 1e9, 1),
                                 "tensor_MB_total": round(sum(4.0 * J for J in Js) / 1e6, 1),
                                 "note": "FP64 FMA tensor pass (4 J R flops per trial) over the whole call's wall "
                                         "time; the 1024 tensors together fit in the 256 MB Infinity Cache"}}


def bench_serving(dgn, torch, n_req=2000, rate=2000.0, slots=8, seed=5):
    """Poisson arrival trace (mean `rate` req/s) of `n_req` distinct seeded fit
    requests, each generated on the GPU before the replay: N in {3,4}, I_n
    log-uniform in [16,256], R ~ U{2..20}, correlation U[0,0.95], 20 dB, 20 %
    complex64 requests, tensors capped at 2^27 entries (larger draws are
    redrawn); stop at |delta eps| < 1e-8 or 200 trials.  The trace runs through
    the server with `slots` concurrent slots plus the batch lane, and through
    one slot without the lane (FIFO one at a time) at the same arrival times."""
    import numpy as np
    from cpgen import device as cdev
    rng = np.random.default_rng(seed)
    t_gen = time.perf_counter()
    probs = cdev.make_pool(torch, seed * 1000, n_req, max_elems=1 << 27)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t_gen
    tensor_bytes = sum(p.y.numel() * p.y.element_size() for p in probs)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    budget = 8 << 30

    def run(nslots, lane):
        srv = dgn.Server(0, budget_bytes=budget, max_slots=nslots, options=dgn.opts(serve_batch=int(lane)))
        facs = [dgn.to_device_factors(p.init) for p in probs]
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        for j, p in enumerate(probs):
            target = t_wall + float(arrivals[j])
            while time.perf_counter() < target:
                pass
            srv.submit(p.y, p.dims, p.R, facs[j], -1.0, 1e-8, 200, tag=j)
        srv.wait_idle()
        res = srv.poll(max_results=n_req)
        srv.close()
        del facs
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        lane_mask = np.array([r["lane"] == 1 for r in res])
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        ok = sum(r["status"] == 0 for r in res)
        out = {"completed": len(res), "ok": int(ok), "fits_per_s": round(len(res) / span, 2),
               "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
               "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
               "span_s": round(span, 3), "trials_total": int(sum(r["info"]["iters"] for r in res))}
        if lane_mask.any():
            sizes = [r["batch_size"] for r in res if r["lane"] == 1]
            out["lane_requests"] = int(lane_mask.sum())
            out["lane_mean_batch"] = round(float(np.mean(sizes)), 1)
            out["lane_p50_latency_ms"] = round(float(np.percentile(lat[lane_mask], 50)) * 1e3, 2)
            out["slot_p50_latency_ms"] = round(float(np.percentile(lat[~lane_mask], 50)) * 1e3, 2)
        return out

    multi = run(slots, True)
    single = run(1, False)
    ncomplex = int(sum(p.complex_ for p in probs))
    del probs
    torch.cuda.empty_cache()
    return {"requests": n_req, "distinct": n_req, "complex_requests": ncomplex, "offered_rate_per_s": rate,
            "slots": slots, "served": multi, "fifo_one_slot": single,
            "speedup_vs_fifo": round(multi["fits_per_s"] / single["fits_per_s"], 2),
            "generation_s": round(gen_s, 1), "tensor_GB": round(tensor_bytes / 1e9, 1),
            "trace": f"Poisson arrivals at {rate:g}/s of {n_req} distinct seeded fits generated on the GPU, "
                     "N in {3,4}, I_n log-uniform [16,256] (tensors <= 2^27 entries), R in [2,20], 20% complex64; "
                     "served = slots + batch lane, fifo = one slot, no lane"}


def bench_als(dgn, torch, ctx, y, dims, R, p, dev, sweeps=5):
    """ALS warm-up sweeps (eq. ALS) on the workload's FP32 tensor: each mode
    update runs one all-mode tensor pass, so a sweep is N passes plus N small
    R x R inversions.  The per-sweep time is the difference of a 1-sweep and a
    `sweeps`-sweep call (both also copy the factors and evaluate the error once)."""
    def timed(k):
        A = dgn.to_device_factors(p.init, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = ctx.cp_als(y, dims, R, A, k)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e
    A = dgn.to_device_factors(p.init, dev)
    e0 = ctx.cp_als(y, dims, R, A, 0)
    timed(1)
    t1, _ = timed(1)
    tk, ek = timed(sweeps)
    per = (tk - t1) / (sweeps - 1)
    ynorm2 = float(torch.sum(y.double() ** 2))
    return {"sweeps": sweeps, "ms_per_sweep": round(per * 1e3, 4), "sweeps_per_s": round(1.0 / per, 2),
            "passes_per_sweep": len(dims), "eps_start": (e0 / ynorm2) ** 0.5, "eps_after": (ek / ynorm2) ** 0.5}


def bench_svd_init(dgn, torch, y, dims, R, dev, block=48, iters=30, reps=3, sample=(200, 200, 200)):
    """SVD initialisation (Section 4.5) of the workload's FP32 tensor: cp_svd_init
    end to end, and its dominant kernel, the three FP64 mode Grams Y_(n) Y_(n)^T on
    the matrix cores, against the FP64 MFMA peak.  Algorithmic flops of a Gram:
    I_n (I_n + 1) K_n (the lower triangle, 2 flops per product, K_n = J / I_n).
    The oracle (a library SVD of every unfolding) is timed on the CPU on a
    `sample`-sized FP64 tensor, with the GPU timed on the same sample."""
    import numpy as np
    from cpgen import synth
    J = 1
    for I in dims:
        J *= I
    rng = np.random.default_rng(8)
    omega = torch.from_numpy(synth.svd_start_block(rng, dims, block)).to(dev)
    ctx = dgn.Context(0, dgn.workspace_size_svd(dims, R, block, y.dtype))
    try:
        ctx.cp_svd_init(y, dims, R, block, omega, iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            A, sv = ctx.cp_svd_init(y, dims, R, block, omega, iters)
        torch.cuda.synchronize()
        init_ms = (time.perf_counter() - t0) / reps * 1e3
        # the three mode Grams alone, HIP events on the stream they run on
        for n in range(len(dims)):
            ctx.mode_gram(y, dims, n)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            for n in range(len(dims)):
                ctx.mode_gram(y, dims, n)
        e1.record()
        torch.cuda.synchronize()
        gram_ms = e0.elapsed_time(e1) / reps
        # the paper's practical start: SVD factors, a few ALS sweeps, then the fit
        # (the same 20 trials as the main line, which starts from random factors)
        fit_ctx = dgn.Context(0, dgn.workspace_size(dims, R, y.dtype) + (64 << 20))
        try:
            info_svd = fit_ctx.cp_fit(y, dims, R, A, -1.0, 0.0, 20, dgn.opts(als_sweeps=3))
        finally:
            fit_ctx.close()
    finally:
        ctx.close()
    flops = sum(I * (I + 1) * (J // I) for I in dims)
    tf = flops / (gram_ms * 1e-3) / 1e12
    # the same init on the bounded sample, GPU and oracle
    from oracle import cp
    ys = synth.cp_tensor([rng.standard_normal((I, R)) for I in sample], 10.0 ** (-np.arange(R) / R))
    ys, _ = synth.add_noise(rng, ys, 25.0)
    yd = torch.from_numpy(ys).to(dev)
    oms = torch.from_numpy(synth.svd_start_block(rng, sample, block)).to(dev)
    c2 = dgn.Context(0, dgn.workspace_size_svd(sample, R, block))
    try:
        c2.cp_svd_init(yd, sample, R, block, oms, iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c2.cp_svd_init(yd, sample, R, block, oms, iters)
        torch.cuda.synchronize()
        gpu_sample_ms = (time.perf_counter() - t0) * 1e3
    finally:
        c2.close()
    Ys = cp.as_tensor(ys, sample)
    t0 = time.perf_counter()
    cp.svd_init(Ys, R)
    cpu_sample_ms = (time.perf_counter() - t0) * 1e3
    return {"block": block, "iters": iters, "ms_per_init": round(init_ms, 3),
            "mode_gram_ms": round(gram_ms, 3),
            "roofline_mode_gram": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK_FP64_TFLOPS,
                                   "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None,
                                   "algorithmic_flops": flops},
            "sample": "x".join(map(str, sample)) + " FP64",
            "fit_from_svd": {"als_sweeps": 3, "trials": info_svd["iters"], "accepted": info_svd["accepted"],
                             "eps": info_svd["eps"]},
            "sample_gpu_ms": round(gpu_sample_ms, 3), "sample_oracle_ms": round(cpu_sample_ms, 1),
            "oracle_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))}


def bench_dgn_vs_flm(dgn, torch, ranks=(5, 10, 20, 30, 40, 50, 60, 64), reps=3, mu=10.0):
    """Time per step and workspace of the fast step (dgn_step) against the plain
    dGN step with J^T J formed explicitly (dgn_step_explicit) on 100 x 100 x 100
    tensors with random entries, as in the paper's complexity study (Section 6),
    for ranks up to this library's limit of 64.  Both steps include the two
    tensor passes (before and after) of a trial."""
    dims = (100, 100, 100)
    J = 100 ** 3
    out = []
    g = torch.Generator(device="cuda")
    for R in ranks:
        g.manual_seed(1000 + R)
        y = torch.randn(J, generator=g, device="cuda", dtype=torch.float64)
        A = [torch.randn((R, 100), generator=g, device="cuda", dtype=torch.float64) for _ in dims]
        ws_f = dgn.workspace_size(dims, R)
        ws_e = dgn.workspace_size_explicit(dims, R)
        ctx = dgn.Context(0, max(ws_f, ws_e) + (16 << 20))
        row = {"R": R, "flm_workspace_MB": round(ws_f / 1e6, 1), "dgn_workspace_MB": round(ws_e / 1e6, 1)}
        try:
            for name, fn in (("flm", ctx.dgn_step), ("dgn", ctx.dgn_step_explicit)):
                fn(y, dims, R, A, mu)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn(y, dims, R, A, mu)
                torch.cuda.synchronize()
                row[f"{name}_ms_per_step"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
        finally:
            ctx.close()
        row["dgn_over_flm_time"] = round(row["dgn_ms_per_step"] / row["flm_ms_per_step"], 2)
        out.append(row)
        del y, A
        torch.cuda.empty_cache()
    return {"tensor": "100x100x100 FP64, random entries", "mu": mu, "steps": out}


def dgn_fit_explicit(ctx, y, dims, R, A0, mu0, tol, max_iters, ynorm2):
    """The plain dGN fit the paper compares with: the damping loop of Section 4.5
    (accept iff the residual decreases, mu <- mu max(1/3, 1 - (2 rho - 1)^3),
    mu <- 2 mu on a rejection, stop on |eps_prev - eps| < tol) driven from the
    host around dgn_step_explicit, whose J^T J is formed and factorised
    explicitly.  A trial whose J^T J + mu I meets a non-positive pivot is
    rejected, as in cp_fit.  No normalisation between trials (the angles of the
    factors do not depend on it)."""
    import math
    import torch
    from paper_1205_2584_amd import dgn
    A = [a.clone() for a in A0]
    B = [torch.empty_like(a) for a in A0]
    mu, eps, it, acc = mu0, None, 0, 0
    while it < max_iters:
        it += 1
        try:
            _, info = ctx.dgn_step_explicit(y, dims, R, A, mu, out=B)
        except dgn.DgnError as e:
            if e.status != -3:
                raise
            # J^T J + mu I not positive definite in FP64: rejected, as cp_fit does
            mu *= 2.0
            continue
        e_old, e_new = info["err2_old"], info["err2_new"]
        if eps is None:
            eps = math.sqrt(e_old / ynorm2)
        if not math.isfinite(e_new):
            break
        if e_new < e_old:
            acc += 1
            rho = (e_old - e_new) / info["denom"]
            A, B = B, A
            eps_prev, eps = eps, math.sqrt(e_new / ynorm2)
            mu *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            if abs(eps_prev - eps) < tol:
                break
        else:
            mu *= 2.0
        if mu > 1e30:
            break
    return A, {"iters": it, "accepted": acc, "eps": eps}


def bench_medsae(dgn, torch, ranks=(5, 10, 20, 30, 40, 60), tensors=2, noisy=2, nu=0.5, snr_db=30.0,
                 tol=1e-8, max_iters=1000, seed=61):
    """Recovery of collinear components by the fast fit (cp_fit) and the plain
    dGN fit (dgn_fit_explicit) on the Section 6.1 data: 100 x 100 x 100 tensors
    of the nu-collinear generator (nu = 0.5: 27 and 37 degrees between
    components) at 30 dB, both fits started from the same mode-n singular
    vectors (cp_svd_init) and the same mu0 (the tau rule), stopped on
    |eps_prev - eps| < 1e-8 or after 1000 trials.  MedSAE (eq. (equ_MedSAE))
    over tensors x noisy runs per rank (the paper: 10 x 20), with the averages
    it plots: first components, and components r >= 2."""
    import numpy as np
    from cpgen import synth
    from paper_1205_2584_amd import metrics
    dims = (100, 100, 100)
    rng = np.random.default_rng(seed)
    out = []
    for R in ranks:
        a2 = {"flm": [], "dgn": []}
        row = {"R": R, "runs": tensors * noisy, "flm": {"iters": [], "eps": [], "s": []},
               "dgn": {"iters": [], "eps": [], "s": []}}
        block = min(80, R + 20)
        ws = max(dgn.workspace_size(dims, R), dgn.workspace_size_explicit(dims, R),
                 dgn.workspace_size_svd(dims, R, block))
        ctx = dgn.Context(0, ws + (16 << 20))
        try:
            for t in range(tensors):
                truth, _ = synth.nu_collinear_factors(rng, dims, R, nu)
                y0 = synth.cp_tensor(truth)
                for k in range(noisy):
                    yn, _ = synth.add_noise(rng, y0, snr_db)
                    y = torch.from_numpy(yn).cuda()
                    ynorm2 = float(np.sum(yn * yn))
                    omega = torch.from_numpy(synth.svd_start_block(rng, dims, block)).cuda()
                    A0, _ = ctx.cp_svd_init(y, dims, R, block, omega, 30)
                    A = [a.clone() for a in A0]
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    fi = ctx.cp_fit(y, dims, R, A, -1.0, tol, max_iters)
                    torch.cuda.synchronize()
                    row["flm"]["s"].append(time.perf_counter() - t0)
                    row["flm"]["iters"].append(fi["iters"])
                    row["flm"]["eps"].append(fi["eps"])
                    a2["flm"].append(metrics.squared_angular_errors(truth, dgn.to_host_factors(A)))
                    t0 = time.perf_counter()
                    B, di = dgn_fit_explicit(ctx, y, dims, R, A0, fi["mu0"], tol, max_iters, ynorm2)
                    torch.cuda.synchronize()
                    row["dgn"]["s"].append(time.perf_counter() - t0)
                    row["dgn"]["iters"].append(di["iters"])
                    row["dgn"]["eps"].append(di["eps"])
                    a2["dgn"].append(metrics.squared_angular_errors(truth, dgn.to_host_factors(B)))
                    print(f"medsae R={R} run={t * noisy + k} flm iters={fi['iters']} eps={fi['eps']:.4e} "
                          f"dgn iters={di['iters']} eps={di['eps']:.4e}", file=sys.stderr, flush=True)
                    del y, A, A0, B
        finally:
            ctx.close()
        for m in ("flm", "dgn"):
            r = row[m]
            r.update(metrics.medsae_summary(a2[m]))
            r["median_iters"] = int(np.median(r.pop("iters")))
            r["median_eps"] = float(np.median(r.pop("eps")))
            s = r.pop("s")
            r["s_per_fit"] = round(float(np.mean(s)), 3)
            r["ms_per_trial"] = round(1e3 * float(np.sum(s)) / max(1, r["median_iters"] * len(s)), 3)
        out.append(row)
        torch.cuda.empty_cache()
    return {"tensor": "100x100x100 FP64, nu-collinear factors (nu = %.2g), %g dB" % (nu, snr_db),
            "init": "mode-n singular vectors", "tol": tol, "max_iters": max_iters, "ranks": out}


def bench_chol_yardstick(torch, sizes, reps=10, seed=21):
    """Library yardstick for factor_solve: torch.linalg.cholesky_ex and
    torch.cholesky_solve (ROCm's dense solver underneath) on seeded SPD FP64
    matrices of the sizes the step factors, timed with events on torch's stream."""
    out = {}
    g = torch.Generator(device="cuda").manual_seed(seed)
    for n in sizes:
        a = torch.randn(n, n, generator=g, device="cuda", dtype=torch.float64)
        s = a @ a.T / n + torch.eye(n, device="cuda", dtype=torch.float64)
        b = torch.randn(n, 1, generator=g, device="cuda", dtype=torch.float64)

        def once():
            L, info = torch.linalg.cholesky_ex(s)
            return torch.cholesky_solve(b, L), info

        for _ in range(3):
            once()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            x, info = once()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[str(n)] = {"ms": round(ms, 4), "TFLOPs": round(n ** 3 / 3 / (ms * 1e-3) / 1e12, 3),
                       "rel_residual": float(torch.linalg.norm(s @ x - b) / torch.linalg.norm(b)),
                       "info": int(info)}
        del a, s, b, x
    return out


def rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_check(dgn, torch, p, ref, mu):
    """Full-size agreement with the FP64 oracle's first step at the initial
    factors: MTTKRP from the FP64, FP32 and BF16 tensors (relative error over
    all modes, against the MTTKRP of the FP64 tensor) and the FP64 step."""
    import numpy as np
    y64 = torch.from_numpy(p.y).cuda()
    ctx = dgn.Context(0, dgn.workspace_size(p.dims, p.R, torch.float64) + (64 << 20))
    out = {}
    Mref = np.concatenate([m.ravel(order="F") for m in ref.M])
    for name, y in (("f64", y64), ("f32", y64.float()), ("bf16", y64.to(torch.bfloat16))):
        M, _ = ctx.dgn_mttkrp(y, p.dims, p.R, dgn.to_device_factors(p.init))
        got = np.concatenate([m.ravel(order="F") for m in dgn.to_host_factors(M)])
        out[f"mttkrp_rel_err_{name}"] = rel(got, Mref)
        del y
    dref = np.concatenate([d.ravel(order="F") for d in ref.dA])
    y32 = y64.float()
    # the first step from each stored precision against the oracle's FP64 step:
    # FP64 tensor; FP32 tensor with the plain pass and with the residual-corrected
    # pass; the FP32 tensor with its BF16 copy for the plain pass
    for name, y, o in (("f64", y64, None), ("f32", y32, None), ("f32_resid", y32, dgn.opts(resid_switch=-1.0)),
                       ("bf16", y32, dgn.opts(y_bf16=y32.to(torch.bfloat16)))):
        A_out, info = ctx.dgn_step(y, p.dims, p.R, dgn.to_device_factors(p.init), mu, o)
        da = np.concatenate([(g - a).ravel(order="F") for g, a in zip(dgn.to_host_factors(A_out), p.init)])
        out[f"step_rel_err_{name}"] = rel(da, dref)
    out["mu"] = mu
    ctx.close()
    del y64, y32
    torch.cuda.empty_cache()
    return out


def precision_oracle_sample(dgn, torch, dims=(150, 150, 150), R=10, trials=150, seed=33):
    """Final eps of the FP64, FP32 and FP32+BF16 paths against the FP64 oracle's fit
    on a sample of the same recipe small enough for the oracle (150^3, R = 10,
    lambda over three decades, correlation 0.9 in mode 3, 25 dB; random start,
    150 trials, no early stop: the oracle reaches the noise floor).  The mixed
    paths are compared with the oracle run on the FP32-rounded tensor."""
    import numpy as np
    import cpgen
    from oracle import cp
    p = cpgen.cfg3(seed=seed, dims=dims, R=R)
    y32h = p.y.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    ref = {"f64": cp.fit(cp.as_tensor(p.y, dims), p.init, mu0=-1.0, tol=0.0, max_iters=trials),
           "f32": cp.fit(cp.as_tensor(y32h, dims), p.init, mu0=-1.0, tol=0.0, max_iters=trials)}
    oracle_s = time.perf_counter() - t0
    y64 = torch.from_numpy(p.y).cuda()
    y32 = y64.float()
    ctx = dgn.Context(0, dgn.workspace_size(dims, R, torch.float64) + (64 << 20))
    out = {"sample": f"{'x'.join(map(str, dims))}, R={R}, {trials} trials from a random start",
           "oracle_s": round(oracle_s, 1)}
    for name, y, o, rk in (("f64", y64, dgn.opts(), "f64"), ("f32", y32, dgn.opts(), "f32"),
                           ("bf16", y32, dgn.opts(y_bf16=y32.to(torch.bfloat16)), "f32")):
        A = dgn.to_device_factors(p.init)
        fi = ctx.cp_fit(y, dims, R, A, -1.0, 0.0, trials, o)
        out[name] = {"eps": fi["eps"], "oracle_eps": ref[rk]["eps"], "eps_diff_vs_oracle": abs(fi["eps"] - ref[rk]["eps"]),
                     "resid_iters": fi["resid_iters"], "accepted": fi["accepted"], "oracle_accepted": ref[rk]["accepted"]}
    ctx.close()
    del y64, y32
    torch.cuda.empty_cache()
    return out


def precision_report(dgn, torch, p):
    """The same fit run for 200 trials with no early stop from the FP64, FP32
    and BF16 tensors (the mixed paths switch to the residual form of the error
    near convergence), so that each path reaches the accuracy it can resolve.
    Reports each final eps and its difference from the FP64 path's.  (With a
    stop test |delta eps| < 1e-8 the FP32 path's stopping point is set by the
    noise of its FP32 residual, about 3e-10 ||Y||^2 in eps^2, and can come early.)
    The comparison with the oracle itself runs on a smaller sample of the recipe
    (precision_oracle_sample)."""
    y64 = torch.from_numpy(p.y).cuda()
    y32 = y64.float()
    ybf = y32.to(torch.bfloat16)
    ctx = dgn.Context(0, dgn.workspace_size(p.dims, p.R, torch.float64) + (64 << 20))
    res = {}
    for name, y, o in (("f64", y64, dgn.opts()), ("f32", y32, dgn.opts()), ("bf16", y32, dgn.opts(y_bf16=ybf))):
        A = dgn.to_device_factors(p.init)
        fi = ctx.cp_fit(y, p.dims, p.R, A, -1.0, 0.0, 200, o)
        res[name] = {"eps": fi["eps"], "iters": fi["iters"], "accepted": fi["accepted"],
                     "reason": fi["reason"], "resid_iters": fi["resid_iters"]}
    ctx.close()
    for name in ("f32", "bf16"):
        res[name]["eps_diff_vs_f64"] = abs(res[name]["eps"] - res["f64"]["eps"])
    del y64, y32, ybf
    torch.cuda.empty_cache()
    res["vs_oracle"] = precision_oracle_sample(dgn, torch)
    return res


def copy_probe(torch, mib):
    """A plain streaming copy of known size: reads `mib` MiB once and writes `mib`
    MiB once (FP32 multiply by one), so that HBM byte counters taken over this
    process can be scaled against a kernel whose traffic is known exactly."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, device="cuda")
    z = torch.empty_like(x)
    torch.mul(x, 1.0, out=z)
    torch.cuda.synchronize()
    del x, z


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="500cube_r30")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-als", action="store_true")
    ap.add_argument("--no-dgn-sweep", action="store_true")
    ap.add_argument("--no-svd", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-hsolve", action="store_true")
    ap.add_argument("--medsae", default="1x1",
                    help="collinear-recovery leg: TENSORSxNOISY runs per rank (0 to skip)")
    ap.add_argument("--only", choices=["batched", "serving", "medsae", "dgn-sweep"], default=None,
                    help="run this leg alone and print its JSON (profiling)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for {args.gpus}); the path is not "
              "sharded across GPUs.", file=sys.stderr)
        raise SystemExit(2)

    import numpy as np
    import torch

    from paper_1205_2584_amd import dgn

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib > 0:
        copy_probe(torch, args.copy_probe_mib)
    if args.only is not None:
        if args.only == "batched":
            leg = bench_batched(dgn, torch)
        elif args.only == "serving":
            leg = bench_serving(dgn, torch)
        elif args.only == "dgn-sweep":
            leg = bench_dgn_vs_flm(dgn, torch)
        else:
            nt, nn = (int(v) for v in (args.medsae if args.medsae != "0" else "1x1").split("x"))
            leg = bench_medsae(dgn, torch, tensors=nt, noisy=nn)
        print(json.dumps({args.only: leg}), flush=True)
        return
    t_gen = time.perf_counter()
    p = workload(args.workload)
    y32 = torch.from_numpy(p.y.astype(np.float32)).to(dev)
    ybf = y32.to(torch.bfloat16)
    dims, R, N = p.dims, p.R, len(p.dims)
    J = int(np.prod(dims))
    gen_s = time.perf_counter() - t_gen
    ws = dgn.workspace_size(dims, R, torch.float32)
    ctx = dgn.Context(0, ws + (64 << 20))

    def run(K, opts):
        A = dgn.to_device_factors(p.init, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.cp_fit(y32, dims, R, A, -1.0, 0.0, K, opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, info

    # FP32 tensor pass (MTTKRP in FP32 with FP32 accumulation), FP64 solve; the
    # rate is taken without per-phase events, the phase times from a second run
    # of the same trials with them
    progress("main fit")
    run(args.warmup, dgn.opts())
    dt, info = run(args.steps, dgn.opts())
    o32 = dgn.opts(timing=1)
    dt_timed, _ = run(args.steps, o32)
    phases, ntr = ctx.dgn_last_phase_times()
    iters = info["iters"]
    per = {k: v / max(ntr, 1) for k, v in phases.items()}
    # BF16 copy for the tensor pass (same solve), reported beside it
    obf = dgn.opts(timing=1, y_bf16=ybf)
    run(args.warmup, obf)
    dtb, infob = run(args.steps, obf)
    phb, ntb = ctx.dgn_last_phase_times()
    perb = {k: v / max(ntb, 1) for k, v in phb.items()}
    # the same fit with the iterative NR^2 solve (CG on the structured SPD
    # system, the direct Cholesky where CG does not converge), reported beside it
    cg_leg = None
    if not args.no_cg:
        ocg = dgn.opts(timing=1, solver=1)
        run(args.warmup, ocg)
        dtc, infoc = run(args.steps, ocg)
        phc, ntc = ctx.dgn_last_phase_times()
        perc = {k: v / max(ntc, 1) for k, v in phc.items()}
        cg_leg = {"iters_per_s": round(infoc["iters"] / dtc, 3), "ms_per_step": round(dtc / max(infoc["iters"], 1) * 1e3, 4),
                  "cg_trials": infoc["cg_trials"], "trials": infoc["iters"],
                  "cg_iters_per_solve": round(infoc["cg_iters"] / max(infoc["cg_trials"], 1), 1),
                  "solve_ms": round(perc["assemble"] + perc["factor_solve"], 4),
                  "direct_solve_ms": round(per["assemble"] + per["factor_solve"], 4),
                  "eps": infoc["eps"], "eps_direct": info["eps"],
                  "phase_ms": {k: round(v, 4) for k, v in perc.items()}}

    pass_ms = per["tensor_pass"]
    pass_gbs = J * 4 / (pass_ms * 1e-3) / 1e9
    passb_gbs = J * 2 / (perb["tensor_pass"] * 1e-3) / 1e9
    fs_ms = per["factor_solve"]
    fs_tf = chol_flops(N, R) / (fs_ms * 1e-3) / 1e12
    upd_tf = schur_update_flops(N, R) / (per["assemble"] * 1e-3) / 1e12
    nr2 = N * R * R
    roof_pass = {"bound": "hbm", "achieved": round(pass_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": round(pass_gbs / PEAK_HBM_GBS, 4), "traffic": traffic("tensor_pass_f32", args.workload),
                 "kernel": "tensor pass: all-mode MTTKRP from one read of the FP32 tensor + slot reductions",
                 "avg_ms": round(pass_ms, 4), "algorithmic_bytes": J * 4}
    roof_sys = {"bound": "mfma", "achieved": round(fs_tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(fs_tf / PEAK_FP64_TFLOPS, 4), "traffic": traffic("factor_solve", args.workload),
                "kernel": "factor_solve: tiled FP64 Cholesky of the (N-1)R^2 Schur complement + substitutions",
                "avg_ms": round(fs_ms, 4), "algorithmic_flops": chol_flops(N, R),
                "assemble_update_TFLOPs": round(upd_tf, 2),
                "dense_lu_equivalent_TFLOPs": round((2.0 / 3.0) * nr2 ** 3 / ((fs_ms + per["assemble"]) * 1e-3) / 1e12, 2)}
    progress("factor_solve yardstick")
    roof_sys["library_yardstick"] = {
        "what": "torch.linalg.cholesky_ex + torch.cholesky_solve on a seeded SPD FP64 matrix of the trailing "
                "system's size (N-1)R^2 and of the whole system's NR^2",
        "ours_ms": round(fs_ms, 4),
        "torch": bench_chol_yardstick(torch, ((N - 1) * R * R, nr2))}
    dominant = roof_sys if fs_ms > pass_ms else roof_pass
    line = {
        "metric": "dGN iters/s at 500^3 R=30 (HBM GB/s); batched CP fits/s + p50/p99 latency",
        "value": round(iters / dt, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": args.warmup,
        "ms_per_step": round(dt / max(iters, 1) * 1e3, 4),
        "ms_per_step_with_phase_events": round(dt_timed / max(iters, 1) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded; truth + 25 dB Gaussian noise)",
        "config": {"workload": f"{'x'.join(map(str, dims))} dense, R={R}, NR^2={N * R * R}",
                   "tensor_pass": "fp32 mttkrp, fp32 accumulation", "solve": "fp64 cholesky"},
        "roofline": dominant,
        "roofline_mttkrp": roof_pass,
        "roofline_solve": roof_sys,
        "phase_ms": {k: round(v, 4) for k, v in per.items()},
        "bf16_pass": {"iters_per_s": round(infob["iters"] / dtb, 3), "tensor_pass_ms": round(perb["tensor_pass"], 4),
                      "tensor_pass_GBs": round(passb_gbs, 1),
                      "roofline": {"bound": "hbm", "achieved": round(passb_gbs, 1), "peak": PEAK_HBM_GBS,
                                   "unit": "GB/s", "frac": round(passb_gbs / PEAK_HBM_GBS, 4),
                                   "traffic": traffic("tensor_pass_bf16", args.workload),
                                   "algorithmic_bytes": J * 2}},
        "fit": {"eps": info["eps"], "accepted": info["accepted"], "mu": info["mu"],
                "resid_iters": info["resid_iters"]},
        "gen_s": round(gen_s, 1),
    }
    if cg_leg is not None:
        line["cg_auto"] = cg_leg
    progress("hessian_solve")
    if not args.no_hsolve:
        # (J^T J + mu I)^-1 V for a random V at the starting factors: the step
        # without its tensor passes (block-form inverse, direct NR^2 solve)
        rng = np.random.default_rng(12)
        A0 = dgn.to_device_factors(p.init, dev)
        V = dgn.to_device_factors([rng.standard_normal((I, R)) for I in dims], dev)
        mu_h = float(info["mu0"])
        ctx.hessian_solve(dims, R, A0, V, mu_h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ctx.hessian_solve(dims, R, A0, V, mu_h)
        torch.cuda.synchronize()
        line["hessian_solve"] = {"ms_per_solve": round((time.perf_counter() - t0) / 5 * 1e3, 4), "mu": mu_h,
                                 "note": "(J^T J + mu I)^-1 V, V random, J at the starting factors of the workload"}
    progress("als")
    if not args.no_als:
        line["als"] = bench_als(dgn, torch, ctx, y32, dims, R, p, dev)
    progress("svd_init")
    if not args.no_svd:
        line["svd_init"] = bench_svd_init(dgn, torch, y32, dims, R, dev)
    ctx.close()
    del y32, ybf
    torch.cuda.empty_cache()
    progress("precision")
    if not args.no_precision:
        line["precision"] = precision_report(dgn, torch, p)
    progress("dgn_vs_flm")
    if not args.no_dgn_sweep:
        line["dgn_vs_flm"] = bench_dgn_vs_flm(dgn, torch)
    progress("medsae")
    if args.medsae != "0":
        nt, nn = (int(v) for v in args.medsae.split("x"))
        line["medsae"] = bench_medsae(dgn, torch, tensors=nt, noisy=nn)
    progress("batched")
    if not args.no_batched:
        line["batched"] = bench_batched(dgn, torch)
    progress("serving")
    if not args.no_serving:
        line["serving"] = bench_serving(dgn, torch)
    progress("cpu_baseline")
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["oracle_check"] = cpu_baseline(p, lambda ref, mu: oracle_check(dgn, torch, p, ref, mu))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
