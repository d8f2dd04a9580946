"""ctypes binding of libdgn.so (C ABI in include/dgn.h), same names as the C calls.

Argument marshalling only: device buffers are torch tensors on a ROCm device,
the stream is torch's current stream.  Factors are float64 tensors of shape
(R, I_n), contiguous -- i.e. column-major I_n x R, the layout the library
expects.  Tensors are 1-D contiguous vec(Y) with the first index fastest.
Every call raises DgnError on a non-zero status; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgn.so")

MAX_ORDER = 8
F64, F32, BF16, C64, C128 = 0, 1, 2, 3, 4
NORM_BALANCED, NORM_UNIT_EXCEPT_LAST, NORM_NONE = 0, 1, 2
MU_PAPER, MU_NIELSEN = 0, 1
BATCH_AUTO, BATCH_GRAPH, BATCH_PERSISTENT = 0, 1, 2
STOP_TOL, STOP_MAX_IT, STOP_MU, STOP_NONFINITE = 0, 1, 2, 3
STATUS = {0: "DGN_OK", -1: "DGN_EINVAL", -2: "DGN_ENOMEM", -3: "DGN_ESINGULAR",
          -4: "DGN_ENONFINITE", -5: "DGN_EHIP", -6: "DGN_EBUSY"}

_DTYPE = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16,
          torch.complex64: C64, torch.complex128: C128}


class DgnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class dgn_tensor(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("dims", ctypes.c_int64 * MAX_ORDER),
                ("dtype", ctypes.c_int32), ("data", ctypes.c_void_p)]


class dgn_opts(ctypes.Structure):
    _fields_ = [("normalize", ctypes.c_int32), ("tau", ctypes.c_double),
                ("resid_switch", ctypes.c_double), ("y_bf16", ctypes.c_void_p),
                ("poll_every", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("als_sweeps", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("cg_max_iters", ctypes.c_int32), ("cg_tol", ctypes.c_double),
                ("mu_rule", ctypes.c_int32), ("batched_launch", ctypes.c_int32),
                ("serve_batch", ctypes.c_int32)]


class dgn_step_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("err2_old", "err2_new", "rho", "denom", "gnorm", "mnorm", "danorm")] + [
        ("cg_iters", ctypes.c_int32), ("cg_attempt_iters", ctypes.c_int32)]


class dgn_fit_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("accepted", ctypes.c_int32), ("reason", ctypes.c_int32),
                ("resid_iters", ctypes.c_int32), ("eps", ctypes.c_double), ("err2", ctypes.c_double),
                ("mu", ctypes.c_double), ("mu0", ctypes.c_double),
                ("cg_trials", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("t_done", ctypes.c_double)]


class dgn_batch_tune_entry(ctypes.Structure):
    _fields_ = [("imax_bucket", ctypes.c_int32), ("rmax", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("us_per_trial_graph", ctypes.c_double), ("us_per_trial_persistent", ctypes.c_double),
                ("sample_fits", ctypes.c_int32), ("sample_trials", ctypes.c_int32)]


class dgn_batch_fit(ctypes.Structure):
    _fields_ = [("Y", dgn_tensor), ("R", ctypes.c_int32), ("mu0", ctypes.c_double),
                ("A", ctypes.c_void_p * 3)]


class dgn_request(ctypes.Structure):
    _fields_ = [("Y", dgn_tensor), ("R", ctypes.c_int32), ("mu0", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("A", ctypes.c_void_p * MAX_ORDER), ("tag", ctypes.c_uint64)]


class dgn_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("info", dgn_fit_info), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("lane", ctypes.c_int32), ("batch_size", ctypes.c_int32)]


EXPORTS = ["dgn_opts_default", "dgn_create", "dgn_destroy", "dgn_last_error", "dgn_workspace_size",
           "dgn_mttkrp", "dgn_step", "dgn_step_explicit", "dgn_workspace_size_explicit", "cp_fit", "cp_als",
           "dgn_mode_gram", "cp_svd_init", "dgn_workspace_size_svd", "dgn_hessian_solve", "dgn_last_phase_times", "cp_fit_batched",
           "dgn_server_create", "dgn_server_submit", "dgn_server_poll", "dgn_server_wait_idle",
           "dgn_server_stats", "dgn_server_now", "dgn_server_destroy", "dgn_step_noalloc",
           "dgn_noalloc_scratch_bytes", "dgn_batched_tuning", "dgn_batched_last_launch"]
NUM_PHASES = 6
PHASES = ["pre", "assemble", "factor_solve", "update", "tensor_pass", "control"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdgn.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.dgn_opts_default.argtypes = [ctypes.POINTER(dgn_opts)]
    L.dgn_opts_default.restype = None
    L.dgn_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_size_t]
    L.dgn_destroy.argtypes = [vp]
    L.dgn_last_error.argtypes = [vp]
    L.dgn_last_error.restype = ctypes.c_char_p
    L.dgn_workspace_size.argtypes = [ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(dgn_opts),
                                     ctypes.POINTER(ctypes.c_size_t)]
    L.dgn_mttkrp.argtypes = [vp, ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(vp),
                             ctypes.POINTER(vp), ctypes.POINTER(dbl), vp]
    L.dgn_step.argtypes = [vp, ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                           dbl, ctypes.POINTER(dgn_opts), ctypes.POINTER(dgn_step_info), vp]
    L.cp_fit.argtypes = [vp, ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(vp), dbl, dbl, i32,
                         ctypes.POINTER(dgn_opts), ctypes.POINTER(dgn_fit_info), vp]
    L.dgn_step_explicit.argtypes = [vp, ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    dbl, ctypes.POINTER(dgn_opts), ctypes.POINTER(dgn_step_info), vp]
    L.dgn_workspace_size_explicit.argtypes = [ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(ctypes.c_size_t)]
    L.cp_als.argtypes = [vp, ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(vp), i32,
                         ctypes.POINTER(dgn_opts), ctypes.POINTER(dbl), vp]
    L.dgn_mode_gram.argtypes = [vp, ctypes.POINTER(dgn_tensor), i32, vp, vp]
    L.dgn_hessian_solve.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), i32, i32, ctypes.POINTER(vp),
                                    ctypes.POINTER(vp), ctypes.POINTER(vp), dbl, ctypes.POINTER(dgn_opts), vp]
    L.cp_svd_init.argtypes = [vp, ctypes.POINTER(dgn_tensor), i32, i32, vp, i32, ctypes.POINTER(vp), vp, vp]
    L.dgn_workspace_size_svd.argtypes = [ctypes.POINTER(dgn_tensor), i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.dgn_last_phase_times.argtypes = [vp, ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]
    L.cp_fit_batched.argtypes = [vp, i32, ctypes.POINTER(dgn_batch_fit), dbl, i32,
                                 ctypes.POINTER(dgn_opts), ctypes.POINTER(dgn_fit_info), vp]
    L.dgn_server_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_size_t, i32, ctypes.POINTER(dgn_opts)]
    L.dgn_server_submit.argtypes = [vp, ctypes.POINTER(dgn_request), ctypes.POINTER(ctypes.c_uint64)]
    L.dgn_server_poll.argtypes = [vp, ctypes.POINTER(dgn_result), i32, ctypes.POINTER(i32)]
    L.dgn_server_wait_idle.argtypes = [vp]
    L.dgn_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.dgn_server_now.argtypes = [vp]
    L.dgn_server_now.restype = dbl
    L.dgn_server_destroy.argtypes = [vp]
    L.dgn_step_noalloc.argtypes = [ctypes.POINTER(dgn_tensor), i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   dbl, ctypes.POINTER(dgn_opts), ctypes.POINTER(dgn_step_info), vp]
    L.dgn_batched_tuning.argtypes = [ctypes.POINTER(dgn_batch_tune_entry), i32, ctypes.POINTER(i32)]
    L.dgn_batched_tuning.restype = ctypes.c_int
    L.dgn_batched_last_launch.argtypes = [vp]
    L.dgn_batched_last_launch.restype = i32
    L.dgn_noalloc_scratch_bytes.argtypes = []
    L.dgn_noalloc_scratch_bytes.restype = ctypes.c_size_t
    for name in ("dgn_create", "dgn_destroy", "dgn_workspace_size", "dgn_mttkrp", "dgn_step", "cp_fit", "cp_als",
                 "dgn_step_explicit", "dgn_workspace_size_explicit",
                 "dgn_mode_gram", "cp_svd_init", "dgn_workspace_size_svd", "dgn_hessian_solve",
                 "dgn_last_phase_times", "cp_fit_batched", "dgn_server_create", "dgn_server_submit",
                 "dgn_server_poll", "dgn_server_wait_idle", "dgn_server_stats", "dgn_server_destroy",
                 "dgn_step_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def tensor_desc(y: torch.Tensor, dims) -> dgn_tensor:
    if y.dim() != 1 or not y.is_contiguous():
        raise ValueError("Y must be a 1-D contiguous tensor holding vec(Y)")
    if y.dtype not in _DTYPE:
        raise ValueError(f"unsupported tensor dtype {y.dtype}")
    J = 1
    for v in dims:
        J *= int(v)
    if y.numel() != J:
        raise ValueError(f"Y holds {y.numel()} elements, the dims need {J}")
    d = dgn_tensor()
    d.order = len(dims)
    for k, v in enumerate(dims):
        d.dims[k] = int(v)
    d.dtype = _DTYPE[y.dtype]
    d.data = y.data_ptr()
    return d


def opts(**kw) -> dgn_opts:
    """dgn_opts with the library defaults and the given fields.  A tensor passed
    as y_bf16 is kept alive by the returned object (the struct holds only its
    device address)."""
    o = dgn_opts()
    load().dgn_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "y_bf16" and isinstance(v, torch.Tensor):
            o._y_bf16 = v
            v = v.data_ptr()
        setattr(o, k, v)
    return o


def _ptrs(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for k, t in enumerate(ts):
        if t.dtype not in (torch.float64, torch.complex128) or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("factors must be contiguous float64 (complex128 for complex tensors) "
                             "device tensors of shape (R, I_n)")
        arr[k] = t.data_ptr()
    return arr


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A dgn_ctx: one device, one workspace arena (allocated once)."""

    def __init__(self, device: int = 0, ws_bytes: int = 0):
        self.L = load()
        h = ctypes.c_void_p()
        st = self.L.dgn_create(ctypes.byref(h), int(device), int(ws_bytes))
        if st != 0:
            raise DgnError(st, "dgn_create failed")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.L.dgn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise DgnError(st, self.L.dgn_last_error(self.h).decode())

    def dgn_mttkrp(self, y, dims, R, factors):
        M = [torch.empty_like(a) for a in factors]
        inner = ctypes.c_double()
        d = tensor_desc(y, dims)
        self._check(self.L.dgn_mttkrp(self.h, ctypes.byref(d), int(R), _ptrs(factors), _ptrs(M),
                                      ctypes.byref(inner), _stream()))
        return M, inner.value

    def dgn_step(self, y, dims, R, factors, mu, options: dgn_opts | None = None, out=None):
        out = [torch.empty_like(a) for a in factors] if out is None else out
        info = dgn_step_info()
        d = tensor_desc(y, dims)
        self._check(self.L.dgn_step(self.h, ctypes.byref(d), int(R), _ptrs(factors), _ptrs(out),
                                    float(mu), ctypes.byref(options) if options else None,
                                    ctypes.byref(info), _stream()))
        return out, {k: getattr(info, k) for k, _ in dgn_step_info._fields_}

    def dgn_step_explicit(self, y, dims, R, factors, mu, options: dgn_opts | None = None, out=None):
        """The plain dGN step with J^T J formed explicitly (same outputs as dgn_step)."""
        out = [torch.empty_like(a) for a in factors] if out is None else out
        info = dgn_step_info()
        d = tensor_desc(y, dims)
        self._check(self.L.dgn_step_explicit(self.h, ctypes.byref(d), int(R), _ptrs(factors), _ptrs(out),
                                             float(mu), ctypes.byref(options) if options else None,
                                             ctypes.byref(info), _stream()))
        return out, {k: getattr(info, k) for k, _ in dgn_step_info._fields_}

    def cp_fit(self, y, dims, R, factors, mu0, tol, max_iters, options: dgn_opts | None = None):
        """Fit in place: `factors` hold the start and receive the result."""
        info = dgn_fit_info()
        d = tensor_desc(y, dims)
        self._check(self.L.cp_fit(self.h, ctypes.byref(d), int(R), _ptrs(factors), float(mu0),
                                  float(tol), int(max_iters),
                                  ctypes.byref(options) if options else None, ctypes.byref(info),
                                  _stream()))
        return {k: getattr(info, k) for k, _ in dgn_fit_info._fields_}

    def cp_als(self, y, dims, R, factors, sweeps, options: dgn_opts | None = None):
        """ALS sweeps in place on `factors`; returns ||Y - Y_hat||^2 after the last one."""
        err2 = ctypes.c_double()
        d = tensor_desc(y, dims)
        self._check(self.L.cp_als(self.h, ctypes.byref(d), int(R), _ptrs(factors), int(sweeps),
                                  ctypes.byref(options) if options else None, ctypes.byref(err2),
                                  _stream()))
        return err2.value

    def hessian_solve(self, dims, R, factors, V, mu, options: dgn_opts | None = None):
        """X = (J^H J + mu I)^-1 vec(V) at the factors; V and the result are (R, I_n)
        float64 (complex128 for complex factors) device tensors (column-major I_n x R blocks)."""
        X = [torch.empty_like(v) for v in V]
        d = (ctypes.c_int64 * len(dims))(*[int(v) for v in dims])
        dt = _DTYPE[torch.complex128] if factors[0].dtype.is_complex else _DTYPE[torch.float64]
        self._check(self.L.dgn_hessian_solve(self.h, len(dims), d, int(R), dt, _ptrs(factors), _ptrs(V), _ptrs(X),
                                             float(mu), ctypes.byref(options) if options else None, _stream()))
        return X

    def mode_gram(self, y, dims, n):
        """Y_(n) Y_(n)^T as an (I_n, I_n) float64 device tensor (enqueued, not synchronised)."""
        d = tensor_desc(y, dims)
        G = None
        if 0 <= int(n) < len(dims):
            gt = torch.complex128 if y.dtype.is_complex else torch.float64
            G = torch.empty((int(dims[n]), int(dims[n])), dtype=gt, device=y.device)
        self._check(self.L.dgn_mode_gram(self.h, ctypes.byref(d), int(n),
                                         ctypes.c_void_p(G.data_ptr() if G is not None else 0), _stream()))
        return G

    def cp_svd_init(self, y, dims, R, block, omega, iters):
        """Leading R left singular vectors of every unfolding; returns (factors, sv):
        factors[n] of shape (R, I_n) (column-major I_n x R; complex128 for complex
        tensors), sv of shape (N, R).  omega: device tensor of sum_n I_n * block
        random start entries (float64, complex128 for complex tensors)."""
        d = tensor_desc(y, dims)
        need = sum(int(I) for I in dims) * int(block)
        ft = torch.complex128 if y.dtype.is_complex else torch.float64
        if omega.dtype != ft or not omega.is_cuda or not omega.is_contiguous() or omega.numel() != need:
            raise ValueError(f"omega must be a contiguous {ft} device tensor of {need} entries")
        A = [torch.empty((int(R), int(I)), dtype=ft, device=y.device) for I in dims]
        sv = torch.empty((len(dims), int(R)), dtype=torch.float64, device=y.device)
        self._check(self.L.cp_svd_init(self.h, ctypes.byref(d), int(R), int(block),
                                       ctypes.c_void_p(omega.data_ptr()), int(iters), _ptrs(A),
                                       ctypes.c_void_p(sv.data_ptr()), _stream()))
        return A, sv

    def cp_fit_batched(self, problems, tol, max_iters, options: dgn_opts | None = None):
        """problems: list of (y, dims, R, factors, mu0); factors are fitted in place.
        Returns one info dict per problem."""
        B = len(problems)
        arr = (dgn_batch_fit * B)()
        for b, (y, dims, R, factors, mu0) in enumerate(problems):
            arr[b].Y = tensor_desc(y, dims)
            arr[b].R = int(R)
            arr[b].mu0 = float(mu0)
            p = _ptrs(factors)
            for n in range(3):
                arr[b].A[n] = p[n]
        infos = (dgn_fit_info * B)()
        self._check(self.L.cp_fit_batched(self.h, B, arr, float(tol), int(max_iters),
                                          ctypes.byref(options) if options else None, infos,
                                          _stream()))
        return [{k: getattr(infos[b], k) for k, _ in dgn_fit_info._fields_} for b in range(B)]

    def batched_last_launch(self):
        """Launch shape (BATCH_GRAPH / BATCH_PERSISTENT) of the last cp_fit_batched call."""
        return int(self.L.dgn_batched_last_launch(self.h))

    def dgn_last_phase_times(self):
        """Per-phase total milliseconds of the last timed cp_fit and the trial count."""
        ms = (ctypes.c_double * NUM_PHASES)()
        n = ctypes.c_int32()
        self._check(self.L.dgn_last_phase_times(self.h, ms, NUM_PHASES, ctypes.byref(n)))
        return dict(zip(PHASES, list(ms))), n.value


def dgn_step_noalloc(y, dims, R, factors, mu, options: dgn_opts | None = None, out=None):
    """dgn_step without a context: the library's fixed per-GPU scratch array is the
    workspace (nothing is allocated on the device).  Runs on the current device."""
    L = load()
    out = [torch.empty_like(a) for a in factors] if out is None else out
    info = dgn_step_info()
    d = tensor_desc(y, dims)
    st = L.dgn_step_noalloc(ctypes.byref(d), int(R), _ptrs(factors), _ptrs(out), float(mu),
                            ctypes.byref(options) if options else None, ctypes.byref(info), _stream())
    if st != 0:
        raise DgnError(st, L.dgn_last_error(None).decode())
    return out, {k: getattr(info, k) for k, _ in dgn_step_info._fields_}


def batched_tuning():
    """The batched tuner's table: one dict per (largest mode size bucket, largest rank) key."""
    out = (dgn_batch_tune_entry * 64)()
    n = ctypes.c_int32()
    st = load().dgn_batched_tuning(out, 64, ctypes.byref(n))
    if st != 0:
        raise DgnError(st, "dgn_batched_tuning failed")
    return [{f: getattr(out[k], f) for f, _ in dgn_batch_tune_entry._fields_} for k in range(n.value)]


def noalloc_scratch_bytes() -> int:
    return int(load().dgn_noalloc_scratch_bytes())


class Server:
    """dgn_server: FIFO admission by device-memory budget, concurrent slots, and
    a batch lane for requests within the batched shapes."""

    def __init__(self, device=0, budget_bytes=1 << 30, max_slots=4, options: dgn_opts | None = None):
        self.L = load()
        h = ctypes.c_void_p()
        st = self.L.dgn_server_create(ctypes.byref(h), int(device), int(budget_bytes), int(max_slots),
                                      ctypes.byref(options) if options else None)
        if st != 0:
            raise DgnError(st, "dgn_server_create failed")
        self.h = h
        self._keep = {}

    def submit(self, y, dims, R, factors, mu0=-1.0, tol=1e-8, max_iters=200, tag=0):
        r = dgn_request()
        r.Y = tensor_desc(y, dims)
        r.R, r.mu0, r.tol, r.max_iters, r.tag = int(R), float(mu0), float(tol), int(max_iters), int(tag)
        p = _ptrs(factors)
        for n in range(len(factors)):
            r.A[n] = p[n]
        rid = ctypes.c_uint64()
        st = self.L.dgn_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid))
        if st != 0:
            raise DgnError(st, "dgn_server_submit failed")
        self._keep[rid.value] = (y, factors)  # the caller's buffers stay alive until polled
        return rid.value

    def poll(self, max_results=256):
        out = (dgn_result * max_results)()
        n = ctypes.c_int32()
        st = self.L.dgn_server_poll(self.h, out, max_results, ctypes.byref(n))
        if st != 0:
            raise DgnError(st, "dgn_server_poll failed")
        res = []
        for k in range(n.value):
            o = out[k]
            self._keep.pop(o.id, None)
            res.append(dict(id=o.id, tag=o.tag, status=o.status,
                            info={f: getattr(o.info, f) for f, _ in dgn_fit_info._fields_},
                            t_submit=o.t_submit, t_admit=o.t_admit, t_done=o.t_done,
                            lane=o.lane, batch_size=o.batch_size))
        return res

    def wait_idle(self):
        self.L.dgn_server_wait_idle(self.h)

    def now(self):
        return self.L.dgn_server_now(self.h)

    def stats(self):
        used, run, q = ctypes.c_size_t(), ctypes.c_int32(), ctypes.c_int32()
        self.L.dgn_server_stats(self.h, ctypes.byref(used), ctypes.byref(run), ctypes.byref(q))
        return used.value, run.value, q.value

    def close(self):
        if self.h:
            self.L.dgn_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size_svd(dims, R, block, dtype=torch.float64) -> int:
    d = dgn_tensor()
    d.order = len(dims)
    for k, v in enumerate(dims):
        d.dims[k] = int(v)
    d.dtype = _DTYPE[dtype]
    d.data = 1
    n = ctypes.c_size_t()
    st = load().dgn_workspace_size_svd(ctypes.byref(d), int(R), int(block), ctypes.byref(n))
    if st != 0:
        raise DgnError(st, "dgn_workspace_size_svd failed")
    return n.value


def workspace_size_explicit(dims, R, dtype=torch.float64) -> int:
    d = dgn_tensor()
    d.order = len(dims)
    for k, v in enumerate(dims):
        d.dims[k] = int(v)
    d.dtype = _DTYPE[dtype]
    d.data = 1
    n = ctypes.c_size_t()
    st = load().dgn_workspace_size_explicit(ctypes.byref(d), int(R), ctypes.byref(n))
    if st != 0:
        raise DgnError(st, "dgn_workspace_size_explicit failed")
    return n.value


def workspace_size(dims, R, dtype=torch.float64) -> int:
    d = dgn_tensor()
    d.order = len(dims)
    for k, v in enumerate(dims):
        d.dims[k] = int(v)
    d.dtype = _DTYPE[dtype]
    d.data = 1
    n = ctypes.c_size_t()
    st = load().dgn_workspace_size(ctypes.byref(d), int(R), None, ctypes.byref(n))
    if st != 0:
        raise DgnError(st, "dgn_workspace_size failed")
    return n.value


# ---- host-side marshalling helpers (numpy <-> device layout) -------------------------

def to_device_factors(A, device="cuda"):
    """numpy (I_n, R) factors -> contiguous (R, I_n) device tensors: float64 for
    real factors, complex128 (interleaved re, im) for complex ones."""
    import numpy as np
    out = []
    for a in A:
        dt = np.complex128 if np.iscomplexobj(a) else np.float64
        out.append(torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=dt).T)).to(device))
    return out


def to_host_factors(ts):
    """(R, I_n) device tensors -> numpy (I_n, R) Fortran-ordered arrays (float64 or complex128)."""
    import numpy as np
    return [np.asfortranarray(t.detach().cpu().numpy().T) for t in ts]
