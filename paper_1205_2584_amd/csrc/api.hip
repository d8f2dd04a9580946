// C ABI of the library (declared in include/dgn.h): argument checking,
// workspace carving and the enqueue order of the kernels of one trial step.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dgn.h"
#include "internal.hpp"

struct dgn_ctx {
  int device;
  char* ws;
  size_t ws_size;
  bool owns_ws = true;
  std::string err;
  std::vector<hipEvent_t> events;   // timing pool, (DGN_NUM_PHASES + 1) per trial
  hipStream_t own = nullptr;        // private stream for graph capture (default priority)
  double phase_ms[DGN_NUM_PHASES] = {0, 0, 0, 0, 0, 0};
  int phase_trials = 0;
  int batch_launch = 0;             // launch shape of the last cp_fit_batched call
};

namespace dgn {
hipError_t launch_inner(const Shape& s, const double* A, const double* M, double* out, hipStream_t st);

// Workspace of cp_fit_batched: a part per fit (its arrays and state) and a
// part per call (the fit table, counters and the launch order); the server's
// batch lane sizes its arena region with these.
size_t batched_ws_fit(const int64_t* dims, int R) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const int I[3] = {(int)dims[0], (int)dims[1], (int)dims[2]};
  return al(batched_fit_doubles(I, R) * sizeof(double)) + al(sizeof(FitState));
}
size_t batched_ws_call(int B) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(sizeof(BFit) * (size_t)B) + al(sizeof(int) * 64) + al(sizeof(int) * (size_t)B);
}

// A context over a caller-provided device region (used by the server's slots).
dgn_ctx* ctx_over(int device, char* ws, size_t size) {
  dgn_ctx* c = new dgn_ctx();
  c->device = device;
  c->ws = ws;
  c->ws_size = size;
  c->owns_ws = false;
  return c;
}
}

namespace {

using namespace dgn;

struct Arena {
  char* base;
  size_t size;
  size_t used = 0;
  bool fail = false;
  template <typename T>
  T* take(size_t n) {
    const size_t bytes = ((n * sizeof(T)) + 255) & ~size_t(255);
    if (used + bytes > size) {
      fail = true;
      used += bytes;
      return nullptr;
    }
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += bytes;
    return p;
  }
};

constexpr int kNormParts = 1024;

// Message of the last failing dgn_step_noalloc call on this thread (no context to hold it).
thread_local std::string g_noalloc_err;

// Launch shapes of cp_fit_batched chosen by its tuner, keyed by the batch's
// largest mode size (in buckets of 16) and largest rank; process-wide.
struct BatchTune {
  int launch;              // DGN_BATCH_GRAPH or DGN_BATCH_PERSISTENT
  double us_graph, us_persistent;
  int sample_fits, sample_trials;
};
std::mutex g_tune_mu;
std::map<std::pair<int, int>, BatchTune> g_tune;

struct Work {
  Shape s;
  YType ymaster;
  int cs = 1;      // doubles per element of the factor / R x R arrays: 1 real, 2 complex
  PassPlan pp;
  SysPlan sp;
  double *A, *Ac, *M, *Mc;
  SmallBuffers sb;
  PassBuffers pb;
  SysBuffers sy;
  SysPlan ep;      // explicit-Hessian system (dgn_step_explicit only)
  SysBuffers ey;
  FitState* state;
  int* flags;      // [0] singular (step), [8..12] CG solve counters (launch_cg), others spare
  double* da_out = nullptr;  // when set, the step's update also writes da (stacked like A)
  int solver = 0;  // dgn_solver
  int cg_max = 0;
  double cg_tol = 0.0;
  double* scr;     // [0..1023] norm partials, [1024] e2, [1025] e2c, [1026..1029] err2 / ynorm2
};

bool dtype_ok(int dt, YType* yt) {
  switch (dt) {
    case DGN_F64: *yt = YType::F64; return true;
    case DGN_F32: *yt = YType::F32; return true;
    case DGN_BF16: *yt = YType::BF16; return true;
    case DGN_C64: *yt = YType::C64; return true;
    case DGN_C128: *yt = YType::C128; return true;
    default: return false;
  }
}

dgn_status set_err(dgn_ctx* ctx, dgn_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

dgn_status check_shape(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, Shape* s, YType* yt) {
  if (!Y) return set_err(ctx, DGN_EINVAL, "tensor descriptor is NULL");
  if (!Y->data) return set_err(ctx, DGN_EINVAL, "tensor data pointer is NULL");
  if (Y->order < 3 || Y->order > DGN_MAX_ORDER)
    return set_err(ctx, DGN_EINVAL, "tensor order must be in [3, 8]");
  if (R < 1 || R > DGN_MAX_RANK) return set_err(ctx, DGN_EINVAL, "rank must be in [1, 64]");
  if (!dtype_ok(Y->dtype, yt))
    return set_err(ctx, DGN_EINVAL, "unsupported tensor dtype");
  if ((*yt == YType::C64 || *yt == YType::C128) && R > kMaxRankC)
    return set_err(ctx, DGN_EINVAL, "complex tensors need rank <= 32");
  s->N = Y->order;
  s->R = R;
  s->T = 0;
  s->maxI = 0;
  long double J = 1;
  for (int n = 0; n < Y->order; ++n) {
    if (Y->dims[n] < 1 || Y->dims[n] > (1LL << 30))
      return set_err(ctx, DGN_EINVAL, "every mode size must be in [1, 2^30]");
    s->I[n] = (int)Y->dims[n];
    s->off[n] = s->T;
    s->T += s->I[n];
    if (s->I[n] > s->maxI) s->maxI = s->I[n];
    J *= (long double)Y->dims[n];
  }
  for (int n = Y->order; n < kMaxOrder; ++n) {
    s->I[n] = 1;
    s->off[n] = s->T;
  }
  if (J > (long double)(1LL << 56)) return set_err(ctx, DGN_EINVAL, "tensor too large");
  return DGN_OK;
}

bool is_complex(YType t) { return t == YType::C64 || t == YType::C128; }

// Pass and system plans for the tensor's type (complex: 32-tiles, embedded system).
void plan(Work& w) {
  w.cs = is_complex(w.ymaster) ? 2 : 1;
  if (w.cs == 2) {
    w.pp = plan_pass_c(w.s);
    w.sp = plan_sys_c(w.s);
  } else {
    w.pp = plan_pass(w.s, w.ymaster);
    w.sp = plan_sys(w.s);
  }
}

void carve(Arena& ar, Work& w, bool with_system) {
  const Shape& s = w.s;
  const size_t cs = (size_t)w.cs;
  const size_t TR = (size_t)s.T * s.R * cs, NR2 = (size_t)s.N * s.R * s.R * cs;
  const int ch = row_chunks(s);
  const size_t stride = (size_t)s.R * s.R * cs + 4;
  w.state = ar.take<FitState>(1);
  w.flags = ar.take<int>(64);
  w.scr = ar.take<double>(kNormParts + 64);
  w.A = ar.take<double>(TR);
  w.Ac = ar.take<double>(TR);
  w.M = ar.take<double>(TR);
  w.Mc = ar.take<double>(TR);
  SmallBuffers& b = w.sb;
  b.C = ar.take<double>(NR2);
  b.Cc = ar.take<double>(NR2);
  b.Gam = ar.take<double>(NR2);
  b.Gt = ar.take<double>(NR2);
  b.X = ar.take<double>(NR2);
  b.Lc = ar.take<double>(NR2);
  b.G = ar.take<double>(TR);
  b.P = ar.take<double>(TR);
  b.wpart = ar.take<double>((size_t)s.N * ch * stride);
  b.rowpart = ar.take<double>((size_t)s.N * ch * stride);
  b.scal = ar.take<double>(8);
  b.ipart = ar.take<double>(((size_t)s.maxI * s.R + 63) / 64);
  b.w = ar.take<double>(NR2);
  b.z = ar.take<double>(NR2);
  b.y = ar.take<double>(NR2);
  b.u = ar.take<double>(NR2);
  b.f = ar.take<double>(NR2);
  b.Q = ar.take<double>(NR2);
  b.Tnm = with_system ? ar.take<double>((size_t)s.N * s.N * s.R * s.R * s.R * cs) : nullptr;
  const PassPlan& p = w.pp;
  const size_t tcb = 8;  // sized for the widest compute type
  w.pb.m0part = ar.take<char>(p.m0_elems * tcb);
  w.pb.m1part = ar.take<char>(p.m1_elems * tcb);
  w.pb.tpart = ar.take<char>(p.t_elems * tcb);
  w.pb.e2part = ar.take<double>(p.e2_elems);
  w.pb.tbuf = p.tbuf_elems ? ar.take<double>(p.tbuf_elems) : nullptr;
  if (with_system) {
    const SysPlan& q = w.sp;
    const size_t r2p = ((size_t)q.R2 + 3) / 4 * 4;
    w.sy.St = ar.take<double>((size_t)q.lds * q.ntp);
    w.sy.B = ar.take<double>((size_t)q.ntp * r2p);
    w.sy.yt = ar.take<double>((size_t)q.ntp);
    w.sy.Ld = ar.take<double>((size_t)q.Tt * 64 * 64);
    w.sy.Li = ar.take<double>((size_t)q.Tt * 64 * 64);
  } else {
    w.sy = SysBuffers{nullptr, nullptr, nullptr, nullptr};
  }
}

dgn_status prepare(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, bool with_system, Work& w) {
  dgn_status st = check_shape(ctx, Y, R, &w.s, &w.ymaster);
  if (st != DGN_OK) return st;
  plan(w);
  Arena ar{ctx ? ctx->ws : nullptr, ctx ? ctx->ws_size : (size_t)-1};
  carve(ar, w, with_system);
  if (ar.fail) {
    return set_err(ctx, DGN_ENOMEM,
                   "workspace budget too small: need " + std::to_string(ar.used) + " bytes, have " +
                       std::to_string(ctx ? ctx->ws_size : 0));
  }
  return DGN_OK;
}

// Workspace of dgn_step_explicit: the small buffers, the tensor pass and the
// RT x RT Hessian system (no fast-step system).
void carve_explicit(Arena& ar, Work& w) {
  carve(ar, w, false);
  w.ep = plan_sys_explicit(w.s);
  const SysPlan& q = w.ep;
  w.ey.St = ar.take<double>((size_t)q.lds * q.ntp);
  w.ey.B = nullptr;
  w.ey.yt = ar.take<double>((size_t)q.ntp);
  w.ey.Ld = ar.take<double>((size_t)q.Tt * 64 * 64);
  w.ey.Li = ar.take<double>((size_t)q.Tt * 64 * 64);
}

dgn_status prepare_explicit(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, Work& w) {
  dgn_status st = check_shape(ctx, Y, R, &w.s, &w.ymaster);
  if (st != DGN_OK) return st;
  if (is_complex(w.ymaster)) return set_err(ctx, DGN_EINVAL, "the explicit-Hessian step is built for real tensors only");
  plan(w);
  Arena ar{ctx ? ctx->ws : nullptr, ctx ? ctx->ws_size : (size_t)-1};
  carve_explicit(ar, w);
  if (ar.fail) {
    return set_err(ctx, DGN_ENOMEM,
                   "workspace budget too small: need " + std::to_string(ar.used) + " bytes, have " +
                       std::to_string(ctx ? ctx->ws_size : 0));
  }
  return DGN_OK;
}

dgn_status hip_fail(dgn_ctx* ctx, hipError_t e, const char* where) {
  return set_err(ctx, DGN_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, where)                       \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

hipError_t copy_factors_in(const Work& w, const void* const* A, double* dst, hipStream_t st) {
  for (int n = 0; n < w.s.N; ++n) {
    hipError_t e = hipMemcpyAsync(dst + (size_t)w.s.off[n] * w.s.R * w.cs, A[n],
                                  sizeof(double) * w.cs * w.s.I[n] * w.s.R, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t copy_factors_out(const Work& w, const double* src, void* const* A, hipStream_t st) {
  for (int n = 0; n < w.s.N; ++n) {
    hipError_t e = hipMemcpyAsync(A[n], src + (size_t)w.s.off[n] * w.s.R * w.cs,
                                  sizeof(double) * w.cs * w.s.I[n] * w.s.R, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The kernels of one trial step from the current (A, M, C) to the candidate
// (Ac, Cc) and the gain-ratio scalars; mu from state when state != NULL.
hipError_t mark(hipEvent_t* ev, int k, hipStream_t st) {
  return ev ? hipEventRecord(ev[k], st) : hipSuccess;
}

// Complex tensors (Section 5): complex small kernels around the real tiled
// Cholesky of the embedded trailing system.
hipError_t enqueue_step_c(Work& w, bool resid, double mu_host, FitState* state, int* singular,
                          const int* stop, hipStream_t st, hipEvent_t* ev) {
  const Shape& s = w.s;
  hipError_t e;
  if ((e = mark(ev, 0, st)) != hipSuccess) return e;
  if ((e = launch_small_pre_c(s, w.A, w.M, resid, mu_host, state, w.sb, singular, stop, st)) != hipSuccess) return e;
  if ((e = mark(ev, 1, st)) != hipSuccess) return e;
  // DGN_SOLVER_AUTO: CG on the Hermitian system first, as in the real step
  const int* solve_stop = stop;
  if (w.solver == DGN_SOLVER_AUTO && cg_supported_c(s)) {
    if ((e = launch_cg_c(s, w.sb, w.cg_tol, w.cg_max, state, mu_host, w.flags + 8, stop, st)) != hipSuccess) return e;
    solve_stop = w.flags + 8;
  }
  if ((e = launch_sys_fill(w.sp, w.sy, solve_stop, st)) != hipSuccess) return e;
  if ((e = launch_subblock_c(s, w.sp, w.sb, w.sy, solve_stop, st)) != hipSuccess) return e;
  if ((e = launch_sys_rhs_syrk(w.sp, w.sb.z, w.sy, solve_stop, st)) != hipSuccess) return e;
  if ((e = mark(ev, 2, st)) != hipSuccess) return e;
  if ((e = launch_sys_factor_solve(s, w.sp, w.sb, w.sy, singular, solve_stop, st)) != hipSuccess) return e;
  if ((e = mark(ev, 3, st)) != hipSuccess) return e;
  return launch_small_post_c(s, w.A, w.Ac, w.sb, mu_host, state, stop, st, w.da_out);
}

// fold_reduce: leave the sums of the update's Gram partials to the tensor pass
// that follows (PassFold); real tensors only.
hipError_t enqueue_step(Work& w, bool resid, double mu_host, FitState* state, int* singular,
                        const int* stop, hipStream_t st, hipEvent_t* ev = nullptr, bool fold_reduce = false) {
  if (w.cs == 2) return enqueue_step_c(w, resid, mu_host, state, singular, stop, st, ev);
  const Shape& s = w.s;
  hipError_t e;
  if ((e = mark(ev, 0, st)) != hipSuccess) return e;
  if ((e = launch_gamma(s, w.sb.C, mu_host, state, w.sb, singular, stop, st)) != hipSuccess) return e;
  if ((e = launch_pw(s, w.A, w.M, resid, w.sb, true, stop, st)) != hipSuccess) return e;
  if ((e = launch_wz(s, w.sb, stop, st)) != hipSuccess) return e;
  if ((e = mark(ev, 1, st)) != hipSuccess) return e;
  // DGN_SOLVER_AUTO: CG first; the direct assembly and solve then skip
  // themselves (flags[8] set) when CG converged or the fit has stopped
  const int* solve_stop = stop;
  if (w.solver == DGN_SOLVER_AUTO && cg_supported(s)) {
    if ((e = launch_cg(s, w.sb, w.cg_tol, w.cg_max, state, mu_host, w.flags + 8, stop, st)) != hipSuccess) return e;
    solve_stop = w.flags + 8;
  }
  if ((e = launch_sys_assemble(s, w.sp, w.sb, w.sy, solve_stop, st)) != hipSuccess) return e;
  if ((e = mark(ev, 2, st)) != hipSuccess) return e;
  if ((e = launch_sys_factor_solve(s, w.sp, w.sb, w.sy, singular, solve_stop, st, s.R <= 32)) != hipSuccess)
    return e;
  if ((e = mark(ev, 3, st)) != hipSuccess) return e;
  if ((e = launch_u(s, w.sb, stop, st)) != hipSuccess) return e;
  if ((e = launch_fq(s, w.sb, stop, st)) != hipSuccess) return e;
  if ((e = launch_update(s, w.A, w.Ac, w.sb, mu_host, state, stop, st, w.da_out)) != hipSuccess) return e;
  if (fold_reduce) return hipSuccess;
  return launch_update_reduce(s, w.sb, w.sb.scal, stop, st);
}

struct PassSel {
  const void* data;
  YType yt;
};

PassSel pass_tensor(const Work& w, const dgn_tensor* Y, const dgn_opts& o, bool resid) {
  if (!resid && w.ymaster == YType::F32 && o.y_bf16) return PassSel{o.y_bf16, YType::BF16};
  return PassSel{Y->data, w.ymaster};
}

hipError_t run_pass(const Work& w, const PassSel& ps, const double* A, bool resid, double* M, double* e2,
                    const int* stop, hipStream_t st, const PassFold* fold = nullptr) {
  if (w.cs == 2)
    return launch_tensor_pass_c(w.s, ps.yt == YType::C128, ps.data, A, resid, w.pp, w.pb, M, e2, stop, st);
  return launch_tensor_pass(w.s, ps.yt, ps.data, A, resid, w.pp, w.pb, M, e2, stop, st, fold);
}

// sum |y|^2; a complex tensor is summed as 2J real values.
hipError_t run_norm2(const PassSel& ps, long long J, double* part, double* out, hipStream_t st) {
  if (ps.yt == YType::C128) return launch_norm2(YType::F64, ps.data, 2 * J, part, kNormParts, out, st);
  if (ps.yt == YType::C64) return launch_norm2(YType::F32, ps.data, 2 * J, part, kNormParts, out, st);
  return launch_norm2(ps.yt, ps.data, J, part, kNormParts, out, st);
}

hipError_t run_gram(const Work& w, const double* A, double* Cout, const int* stop, hipStream_t st) {
  if (w.cs == 2) return launch_gram_c(w.s, A, w.sb, Cout, stop, st);
  return launch_gram(w.s, A, w.sb, Cout, stop, st);
}

// ALS sweeps (eq. ALS) on the workspace factors w.A: modes in turn, each from a
// fresh Gram set, Gamma^(n)^-1 (k_gamma / k_gamma_c at mu = 0) and an all-mode
// tensor pass (with conjugated factors for complex tensors, Theorem 5.4).
// A Gamma^(n) that is not positive definite raises singular[0].
hipError_t enqueue_als(Work& w, const PassSel& plain, int sweeps, int* singular, hipStream_t st) {
  const Shape& s = w.s;
  hipError_t e;
  for (int it = 0; it < sweeps; ++it)
    for (int n = 0; n < s.N; ++n) {
      if ((e = run_gram(w, w.A, w.sb.C, nullptr, st)) != hipSuccess) return e;
      e = (w.cs == 2) ? launch_gamma_c(s, w.sb.C, 0.0, nullptr, w.sb, singular, nullptr, st)
                      : launch_gamma(s, w.sb.C, 0.0, nullptr, w.sb, singular, nullptr, st);
      if (e != hipSuccess) return e;
      if ((e = run_pass(w, plain, w.A, false, w.M, nullptr, nullptr, st)) != hipSuccess) return e;
      e = (w.cs == 2) ? launch_als_rows_c(s, n, w.M, w.sb, w.A, st) : launch_als_rows(s, n, w.M, w.sb, w.A, st);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

}  // namespace

extern "C" {

void dgn_opts_default(dgn_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->normalize = DGN_NORM_BALANCED;
  o->tau = 1e-3;
  o->resid_switch = 1e-3;
  o->y_bf16 = nullptr;
  o->poll_every = 8;
  o->timing = 0;
  o->graph = 1;
  o->solver = DGN_SOLVER_DIRECT;
  o->cg_max_iters = 100;
  o->cg_tol = 1e-10;
  o->mu_rule = DGN_MU_PAPER;
  o->batched_launch = DGN_BATCH_AUTO;
  o->serve_batch = 1;
}

dgn_status dgn_create(dgn_ctx** out, int32_t device, size_t ws_budget_bytes) {
  if (!out) return DGN_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DGN_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return DGN_EHIP;
  dgn_ctx* c = new dgn_ctx();
  c->device = device;
  c->ws_size = ws_budget_bytes ? ws_budget_bytes : (size_t(1) << 30);
  if (hipMalloc((void**)&c->ws, c->ws_size) != hipSuccess) {
    delete c;
    return DGN_ENOMEM;
  }
  *out = c;
  return DGN_OK;
}

dgn_status dgn_destroy(dgn_ctx* ctx) {
  if (!ctx) return DGN_EINVAL;
  hipSetDevice(ctx->device);
  for (hipEvent_t e : ctx->events) hipEventDestroy(e);
  if (ctx->own) hipStreamDestroy(ctx->own);
  if (ctx->owns_ws) hipFree(ctx->ws);
  delete ctx;
  return DGN_OK;
}

const char* dgn_last_error(const dgn_ctx* ctx) { return ctx ? ctx->err.c_str() : g_noalloc_err.c_str(); }

dgn_status dgn_last_phase_times(const dgn_ctx* ctx, double* ms_out, int32_t n, int32_t* trials) {
  if (!ctx || (!ms_out && n > 0) || n < 0 || n > DGN_NUM_PHASES) return DGN_EINVAL;
  for (int k = 0; k < n; ++k) ms_out[k] = ctx->phase_ms[k];
  if (trials) *trials = ctx->phase_trials;
  return DGN_OK;
}

dgn_status dgn_workspace_size(const dgn_tensor* Y, int32_t R, const dgn_opts* opts, size_t* bytes) {
  (void)opts;
  if (!bytes) return DGN_EINVAL;
  Work w{};
  dgn_status st = check_shape(nullptr, Y, R, &w.s, &w.ymaster);
  if (st != DGN_OK) return st;
  plan(w);
  Arena ar{nullptr, (size_t)-1};
  carve(ar, w, true);
  *bytes = ar.used;
  return DGN_OK;
}

dgn_status dgn_workspace_size_explicit(const dgn_tensor* Y, int32_t R, size_t* bytes) {
  if (!bytes) return DGN_EINVAL;
  Work w{};
  dgn_status st = check_shape(nullptr, Y, R, &w.s, &w.ymaster);
  if (st != DGN_OK) return st;
  if (is_complex(w.ymaster)) return DGN_EINVAL;
  plan(w);
  Arena ar{nullptr, (size_t)-1};
  carve_explicit(ar, w);
  *bytes = ar.used;
  return DGN_OK;
}

dgn_status dgn_mttkrp(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, const void* const* A,
                      void* const* M, double* inner, void* stream) {
  if (!ctx) return DGN_EINVAL;
  if (!A || !M) return set_err(ctx, DGN_EINVAL, "factor or output pointer array is NULL");
  Work w{};
  dgn_status rc = prepare(ctx, Y, R, false, w);
  if (rc != DGN_OK) return rc;
  for (int n = 0; n < w.s.N; ++n)
    if (!A[n] || !M[n]) return set_err(ctx, DGN_EINVAL, "NULL factor or output pointer");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  HIPCHK(copy_factors_in(w, A, w.A, st), "copy factors");
  HIPCHK(run_pass(w, PassSel{Y->data, w.ymaster}, w.A, false, w.M, nullptr, nullptr, st), "tensor pass");
  HIPCHK(copy_factors_out(w, w.M, M, st), "copy MTTKRP");
  if (inner) {
    if (w.cs == 2) HIPCHK(launch_inner_c(w.s, w.A, w.M, w.scr + 1026, st), "inner");
    else HIPCHK(launch_inner(w.s, w.A, w.M, w.scr + 1026, st), "inner");
    HIPCHK(hipMemcpyAsync(inner, w.scr + 1026, sizeof(double), hipMemcpyDeviceToHost, st), "copy inner");
    HIPCHK(hipStreamSynchronize(st), "sync");
  }
  return DGN_OK;
}

}  // extern "C"

namespace {

// Zero n ints on the stream with a kernel (no memset node, so the enqueue
// sequence stays free of hipMemsetAsync).
__global__ void k_zero_ints(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// dgn_step on the workspace of ctx (a context's own arena, or the fixed
// scratch array of dgn_step_noalloc).
dgn_status step_impl(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, const void* const* A_in,
                     void* const* A_out, double mu, const dgn_opts* opts, dgn_step_info* info,
                     void* stream) {
  if (!A_in || !A_out) return set_err(ctx, DGN_EINVAL, "factor pointer array is NULL");
  if (!(mu > 0.0) || !isfinite(mu)) return set_err(ctx, DGN_EINVAL, "mu must be finite and > 0");
  dgn_opts o;
  dgn_opts_default(&o);
  if (opts) o = *opts;
  if (o.solver != DGN_SOLVER_DIRECT && o.solver != DGN_SOLVER_AUTO) return set_err(ctx, DGN_EINVAL, "bad solver option");
  if (o.solver == DGN_SOLVER_AUTO && (o.cg_max_iters < 0 || !(o.cg_tol > 0.0)))
    return set_err(ctx, DGN_EINVAL, "need cg_max_iters >= 0 and cg_tol > 0");
  Work w{};
  dgn_status rc = prepare(ctx, Y, R, true, w);
  if (rc != DGN_OK) return rc;
  for (int n = 0; n < w.s.N; ++n)
    if (!A_in[n] || !A_out[n]) return set_err(ctx, DGN_EINVAL, "NULL factor pointer");
  w.solver = o.solver;
  w.cg_max = o.cg_max_iters;
  w.cg_tol = o.cg_tol;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  const bool resid = (w.ymaster == YType::F64) || w.cs == 2 || o.resid_switch < 0;
  const PassSel ps = pass_tensor(w, Y, o, resid);
  const long long J = [&] { long long j = 1; for (int n = 0; n < w.s.N; ++n) j *= w.s.I[n]; return j; }();
  double* ynp = w.scr + 1028;
  double* e2a = w.scr + 1024;
  double* e2b = w.scr + 1025;
  double* out = w.scr + 1026;  // err2 old, new
  k_zero_ints<<<1, 64, 0, st>>>(w.flags, 64);
  HIPCHK(hipGetLastError(), "zero flags");
  HIPCHK(copy_factors_in(w, A_in, w.A, st), "copy factors");
  HIPCHK(run_norm2(ps, J, w.scr, ynp, st), "norm");
  HIPCHK(run_gram(w, w.A, w.sb.C, nullptr, st), "gram");
  HIPCHK(run_pass(w, ps, w.A, resid, w.M, e2a, nullptr, st), "pass");
  HIPCHK(launch_err2(w.s, w.A, w.M, w.sb.C, resid, e2a, ynp, out, st), "err2");
  HIPCHK(enqueue_step(w, resid, mu, nullptr, w.flags, nullptr, st), "step");
  HIPCHK(run_pass(w, ps, w.Ac, resid, w.Mc, e2b, nullptr, st), "pass");
  HIPCHK(launch_err2(w.s, w.Ac, w.Mc, w.sb.Cc, resid, e2b, ynp, out + 1, st), "err2");
  HIPCHK(copy_factors_out(w, w.Ac, A_out, st), "copy out");
  double host[2] = {0, 0}, sc[4] = {0, 0, 0, 0};
  int flags[16] = {0};
  HIPCHK(hipMemcpyAsync(host, out, sizeof host, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipMemcpyAsync(sc, w.sb.scal, sizeof sc, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  const bool cg_ran = w.solver == DGN_SOLVER_AUTO && (w.cs == 1 ? cg_supported(w.s) : cg_supported_c(w.s));
  if (info) {
    info->cg_iters = (cg_ran && flags[8]) ? flags[10] : -1;
    info->cg_attempt_iters = cg_ran ? flags[10] : -1;
    info->err2_old = host[0];
    info->err2_new = host[1];
    info->denom = sc[0];
    info->rho = (host[0] - host[1]) / sc[0];
    info->danorm = sqrt(sc[1]);
    info->gnorm = sqrt(sc[2]);
    info->mnorm = sqrt(sc[3]);
  }
  if (flags[0]) return set_err(ctx, DGN_ESINGULAR, "non-positive pivot in (Gamma + mu I) or the NR^2 system");
  if (!isfinite(host[1]) || !isfinite(sc[0])) return set_err(ctx, DGN_ENONFINITE, "non-finite step");
  return DGN_OK;
}

// The fixed scratch of dgn_step_noalloc: one array per GPU the library runs
// on (each device holds its own copy at its own address), held until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy: the name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
char* g_scratch_ptr[kNoAllocMaxDevices] = {};

}  // namespace

extern "C" {

dgn_status dgn_step(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, const void* const* A_in,
                    void* const* A_out, double mu, const dgn_opts* opts, dgn_step_info* info,
                    void* stream) {
  if (!ctx) return DGN_EINVAL;
  return step_impl(ctx, Y, R, A_in, A_out, mu, opts, info, stream);
}

size_t dgn_noalloc_scratch_bytes(void) { return kNoAllocBytes; }

dgn_status dgn_step_noalloc(const dgn_tensor* Y, int32_t R, const void* const* A_in, void* const* A_out,
                            double mu, const dgn_opts* opts, dgn_step_info* info, void* stream) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) {
    g_noalloc_err = "dgn_step_noalloc: no usable current device";
    return DGN_EHIP;
  }
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        g_noalloc_err = std::string("dgn_step_noalloc: hipGetSymbolAddress of the scratch array: ") +
                        hipGetErrorString(e);
        return DGN_EHIP;
      }
      g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    base = g_scratch_ptr[dev];
  }
  size_t need = 0;
  dgn_status rc = dgn_workspace_size(Y, R, opts, &need);
  if (rc != DGN_OK) {
    g_noalloc_err = "dgn_step_noalloc: bad tensor descriptor or rank";
    return rc;
  }
  if (need > kNoAllocBytes) {
    g_noalloc_err = "dgn_step_noalloc: this shape needs " + std::to_string(need) +
                    " bytes of scratch, above the fixed maximum of " + std::to_string(kNoAllocBytes) +
                    " bytes; use dgn_step with a context";
    return DGN_ENOMEM;
  }
  dgn_ctx c;  // a context over the scratch array: nothing is allocated on the device
  c.device = dev;
  c.ws = base;
  c.ws_size = kNoAllocBytes;
  c.owns_ws = false;
  rc = step_impl(&c, Y, R, A_in, A_out, mu, opts, info, stream);
  g_noalloc_err = rc == DGN_OK ? std::string() : c.err;
  return rc;
}

dgn_status dgn_hessian_solve(dgn_ctx* ctx, int32_t order, const int64_t* dims, int32_t R, int32_t dtype,
                             const void* const* A, const void* const* V, void* const* X, double mu,
                             const dgn_opts* opts, void* stream) {
  if (!ctx) return DGN_EINVAL;
  if (!dims || !A || !V || !X) return set_err(ctx, DGN_EINVAL, "NULL dims or pointer array");
  if (!(mu > 0.0) || !isfinite(mu)) return set_err(ctx, DGN_EINVAL, "mu must be finite and > 0");
  dgn_opts o;
  dgn_opts_default(&o);
  if (opts) o = *opts;
  if (o.solver != DGN_SOLVER_DIRECT && o.solver != DGN_SOLVER_AUTO) return set_err(ctx, DGN_EINVAL, "bad solver option");
  if (o.solver == DGN_SOLVER_AUTO && (o.cg_max_iters < 0 || !(o.cg_tol > 0.0)))
    return set_err(ctx, DGN_EINVAL, "need cg_max_iters >= 0 and cg_tol > 0");
  if (order < 3 || order > DGN_MAX_ORDER) return set_err(ctx, DGN_EINVAL, "order must be in [3, 8]");
  if (dtype != DGN_F64 && dtype != DGN_C128) return set_err(ctx, DGN_EINVAL, "dtype must be DGN_F64 or DGN_C128");
  // the system depends on the factors only: plan it as for an FP64 (complex128)
  // tensor of these sizes, whose data is never read
  dgn_tensor t{};
  t.order = order;
  for (int n = 0; n < order; ++n) t.dims[n] = dims[n];
  t.dtype = dtype;
  t.data = &t;
  Work w{};
  dgn_status rc = prepare(ctx, &t, R, true, w);
  if (rc != DGN_OK) return rc;
  for (int n = 0; n < w.s.N; ++n)
    if (!A[n] || !V[n] || !X[n]) return set_err(ctx, DGN_EINVAL, "NULL factor or block pointer");
  w.solver = o.solver;
  w.cg_max = o.cg_max_iters;
  w.cg_tol = o.cg_tol;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  HIPCHK(hipMemsetAsync(w.flags, 0, 64 * sizeof(int), st), "memset");
  HIPCHK(copy_factors_in(w, A, w.A, st), "copy factors");
  HIPCHK(copy_factors_in(w, V, w.M, st), "copy right-hand side");
  HIPCHK(run_gram(w, w.A, w.sb.C, nullptr, st), "gram");
  // the step with M taken as the gradient (its residual form) solves
  // (J^T J + mu I) da = vec(V); the update hands da out into Mc
  w.da_out = w.Mc;
  HIPCHK(enqueue_step(w, true, mu, nullptr, w.flags, nullptr, st), "solve");
  HIPCHK(copy_factors_out(w, w.Mc, X, st), "copy out");
  int flags[1] = {0};
  HIPCHK(hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  if (flags[0]) return set_err(ctx, DGN_ESINGULAR, "non-positive pivot in (Gamma + mu I) or the NR^2 system");
  return DGN_OK;
}

dgn_status dgn_step_explicit(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, const void* const* A_in,
                             void* const* A_out, double mu, const dgn_opts* opts, dgn_step_info* info,
                             void* stream) {
  if (!ctx) return DGN_EINVAL;
  if (!A_in || !A_out) return set_err(ctx, DGN_EINVAL, "factor pointer array is NULL");
  if (!(mu > 0.0) || !isfinite(mu)) return set_err(ctx, DGN_EINVAL, "mu must be finite and > 0");
  dgn_opts o;
  dgn_opts_default(&o);
  if (opts) o = *opts;
  Work w{};
  dgn_status rc = prepare_explicit(ctx, Y, R, w);
  if (rc != DGN_OK) return rc;
  for (int n = 0; n < w.s.N; ++n)
    if (!A_in[n] || !A_out[n]) return set_err(ctx, DGN_EINVAL, "NULL factor pointer");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  const Shape& s = w.s;
  const bool resid = (w.ymaster == YType::F64) || o.resid_switch < 0;
  const PassSel ps = pass_tensor(w, Y, o, resid);
  const long long J = [&] { long long j = 1; for (int n = 0; n < s.N; ++n) j *= s.I[n]; return j; }();
  double* ynp = w.scr + 1028;
  double* e2a = w.scr + 1024;
  double* e2b = w.scr + 1025;
  double* out = w.scr + 1026;
  HIPCHK(hipMemsetAsync(w.flags, 0, 64 * sizeof(int), st), "memset");
  HIPCHK(copy_factors_in(w, A_in, w.A, st), "copy factors");
  HIPCHK(run_norm2(ps, J, w.scr, ynp, st), "norm");
  HIPCHK(run_gram(w, w.A, w.sb.C, nullptr, st), "gram");
  HIPCHK(run_pass(w, ps, w.A, resid, w.M, e2a, nullptr, st), "pass");
  HIPCHK(launch_err2(s, w.A, w.M, w.sb.C, resid, e2a, ynp, out, st), "err2");
  // gradient blocks G (and ||G||^2, ||M||^2) through the fast step's own kernels
  HIPCHK(launch_gamma(s, w.sb.C, mu, nullptr, w.sb, w.flags, nullptr, st), "gamma");
  HIPCHK(launch_pw(s, w.A, w.M, resid, w.sb, false, nullptr, st), "pw");
  HIPCHK(launch_wz(s, w.sb, nullptr, st), "wz");
  // (J^T J + mu I) da = g, J^T J formed explicitly
  HIPCHK(launch_explicit_system(s, w.ep, w.A, w.sb.C, w.sb.G, mu, w.ey.St, st), "hessian");
  HIPCHK(launch_sys_factor_solve_core(w.ep, w.ey, w.flags, nullptr, st), "factor");
  HIPCHK(launch_explicit_update(w.ep, w.A, w.ey.yt, w.sb.G, mu, w.Ac, w.sb.scal, st), "update");
  HIPCHK(run_gram(w, w.Ac, w.sb.Cc, nullptr, st), "gram");
  HIPCHK(run_pass(w, ps, w.Ac, resid, w.Mc, e2b, nullptr, st), "pass");
  HIPCHK(launch_err2(s, w.Ac, w.Mc, w.sb.Cc, resid, e2b, ynp, out + 1, st), "err2");
  HIPCHK(copy_factors_out(w, w.Ac, A_out, st), "copy out");
  double host[2] = {0, 0}, sc[4] = {0, 0, 0, 0};
  int flags[1] = {0};
  HIPCHK(hipMemcpyAsync(host, out, sizeof host, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipMemcpyAsync(sc, w.sb.scal, sizeof sc, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  if (info) {
    info->err2_old = host[0];
    info->err2_new = host[1];
    info->denom = sc[0];
    info->rho = (host[0] - host[1]) / sc[0];
    info->danorm = sqrt(sc[1]);
    info->gnorm = sqrt(sc[2]);
    info->mnorm = sqrt(sc[3]);
    info->cg_iters = -1;
    info->cg_attempt_iters = -1;
  }
  if (flags[0]) return set_err(ctx, DGN_ESINGULAR, "non-positive pivot in J^T J + mu I");
  if (!isfinite(host[1]) || !isfinite(sc[0])) return set_err(ctx, DGN_ENONFINITE, "non-finite step");
  return DGN_OK;
}

dgn_status cp_fit(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, void* const* A, double mu0,
                  double tol, int32_t max_iters, const dgn_opts* opts, dgn_fit_info* info,
                  void* stream) {
  if (!ctx) return DGN_EINVAL;
  if (!A) return set_err(ctx, DGN_EINVAL, "factor pointer array is NULL");
  if (max_iters < 0 || !(tol >= 0.0) || !isfinite(mu0))
    return set_err(ctx, DGN_EINVAL, "need max_iters >= 0, tol >= 0 and a finite mu0");
  dgn_opts o;
  dgn_opts_default(&o);
  if (opts) o = *opts;
  if (o.poll_every < 1) o.poll_every = 1;
  if (o.normalize < 0 || o.normalize > 2) return set_err(ctx, DGN_EINVAL, "bad normalize option");
  if (o.mu_rule != DGN_MU_PAPER && o.mu_rule != DGN_MU_NIELSEN) return set_err(ctx, DGN_EINVAL, "bad mu_rule option");
  if (o.als_sweeps < 0) return set_err(ctx, DGN_EINVAL, "als_sweeps must be >= 0");
  if (o.solver != DGN_SOLVER_DIRECT && o.solver != DGN_SOLVER_AUTO) return set_err(ctx, DGN_EINVAL, "bad solver option");
  if (o.solver == DGN_SOLVER_AUTO && (o.cg_max_iters < 0 || !(o.cg_tol > 0.0)))
    return set_err(ctx, DGN_EINVAL, "need cg_max_iters >= 0 and cg_tol > 0");
  Work w{};
  dgn_status rc = prepare(ctx, Y, R, true, w);
  if (rc != DGN_OK) return rc;
  for (int n = 0; n < w.s.N; ++n)
    if (!A[n]) return set_err(ctx, DGN_EINVAL, "NULL factor pointer");
  w.solver = o.solver;
  w.cg_max = o.cg_max_iters;
  w.cg_tol = o.cg_tol;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  HIPCHK(hipMemsetAsync(w.flags, 0, 64 * sizeof(int), st), "memset");
  bool resid = (w.ymaster == YType::F64) || w.cs == 2 || o.resid_switch < 0;
  const bool can_switch = !resid && o.resid_switch > 0;
  PassSel ps = pass_tensor(w, Y, o, resid);
  const long long J = [&] { long long j = 1; for (int n = 0; n < w.s.N; ++n) j *= w.s.I[n]; return j; }();
  FitState hs;
  memset(&hs, 0, sizeof hs);
  hs.tol = tol;
  hs.max_iters = max_iters;
  hs.normalize = o.normalize;
  hs.mu_rule = o.mu_rule;
  hs.stop = 0;
  FitState* ds = w.state;
  double* e2 = w.scr + 1024;
  double* e2c = w.scr + 1025;
  HIPCHK(hipMemcpyAsync(ds, &hs, sizeof hs, hipMemcpyHostToDevice, st), "state");
  HIPCHK(copy_factors_in(w, A, w.A, st), "copy factors");
  if (o.als_sweeps > 0) {  // warm-up on the starting factors (eq. ALS)
    HIPCHK(hipMemsetAsync(w.flags, 0, 64 * sizeof(int), st), "memset");
    HIPCHK(enqueue_als(w, pass_tensor(w, Y, o, false), o.als_sweeps, w.flags, st), "als");
  }
  HIPCHK(run_norm2(PassSel{Y->data, w.ymaster}, J, w.scr, &ds->ynorm2, st), "norm");
  HIPCHK(run_norm2(ps, J, w.scr, &ds->ynorm2_pass, st), "norm");
  HIPCHK(run_gram(w, w.A, w.sb.C, nullptr, st), "gram");
  HIPCHK(run_pass(w, ps, w.A, resid, w.M, e2, nullptr, st), "pass");
  HIPCHK(launch_fit_init(w.s, w.A, w.M, w.sb.C, resid, e2, mu0, o.tau, ds, st, w.cs), "init");
  const int* stop = &ds->stop;
  const int EV = DGN_NUM_PHASES + 1;
  if (o.timing) {
    const size_t need = (size_t)EV * max_iters;
    while (ctx->events.size() < need) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e), "hipEventCreate");
      ctx->events.push_back(e);
    }
  }
  ctx->phase_trials = 0;
  for (int k = 0; k < DGN_NUM_PHASES; ++k) ctx->phase_ms[k] = 0.0;
  int enq = 0;
  for (int t = 0; t < max_iters; ++t) {
    hipEvent_t* ev = o.timing ? &ctx->events[(size_t)EV * t] : nullptr;
    // real tensors: the Gram sums of the update and the pieces of <A_1, M_1>
    // ride in the pass's reduction launch
    const bool fold = w.cs != 2;
    PassFold pf;
    if (fold) {
      pf.ipart = resid ? nullptr : w.sb.ipart;
      pf.rowpart = w.sb.rowpart;
      pf.chunks = row_chunks(w.s);
      pf.stride = w.s.R * w.s.R + 4;
      pf.gout = w.sb.Cc;
      pf.gscal = w.sb.scal;
    }
    HIPCHK(enqueue_step(w, resid, 0.0, ds, &ds->singular, stop, st, ev, fold), "step");
    HIPCHK(mark(ev, 4, st), "event");
    HIPCHK(run_pass(w, ps, w.Ac, resid, w.Mc, e2c, stop, st, fold ? &pf : nullptr), "pass");
    HIPCHK(mark(ev, 5, st), "event");
    HIPCHK(launch_control(w.s, w.Ac, w.Mc, w.sb.Cc, resid, e2c, w.sb.scal, ds, t, st, w.cs, pf.ipart,
                          (int)(((long long)w.s.I[0] * w.s.R + 63) / 64)),
           "control");
    HIPCHK(launch_commit(w.s, w.A, w.Ac, w.M, w.Mc, w.sb.C, w.sb.Cc, ds, t, st, w.cs), "commit");
    HIPCHK(mark(ev, 6, st), "event");
    enq = t + 1;
    if ((t + 1) % o.poll_every == 0 || t + 1 == max_iters) {
      HIPCHK(hipMemcpyAsync(&hs, ds, sizeof hs, hipMemcpyDeviceToHost, st), "poll");
      HIPCHK(hipStreamSynchronize(st), "sync");
      if (hs.stop) break;
      if (can_switch && !resid && hs.accepted > 0 && fabs(hs.eps_prev - hs.eps) < o.resid_switch) {
        resid = true;
        ps = pass_tensor(w, Y, o, resid);
        HIPCHK(run_pass(w, ps, w.A, true, w.M, e2, stop, st), "pass");
        HIPCHK(launch_refresh(w.s, e2, ds, st), "refresh");
      }
    }
  }
  HIPCHK(copy_factors_out(w, w.A, A, st), "copy out");
  HIPCHK(hipMemcpyAsync(&hs, ds, sizeof hs, hipMemcpyDeviceToHost, st), "state");
  int fl[16] = {0};
  HIPCHK(hipMemcpyAsync(fl, w.flags, sizeof fl, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  const int als_flag = o.als_sweeps > 0 ? fl[0] : 0;
  if (als_flag) return set_err(ctx, DGN_ESINGULAR, "a Gamma^(n) of the ALS warm-up is not positive definite");
  if (o.timing) {
    const int nt = hs.iters < enq ? hs.iters : enq;
    for (int t = 0; t < nt; ++t) {
      for (int k = 0; k < DGN_NUM_PHASES; ++k) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->events[(size_t)EV * t + k], ctx->events[(size_t)EV * t + k + 1]),
               "hipEventElapsedTime");
        ctx->phase_ms[k] += ms;
      }
    }
    ctx->phase_trials = nt;
  }
  if (info) {
    info->iters = hs.iters;
    info->accepted = hs.accepted;
    info->reason = hs.reason;
    info->resid_iters = hs.resid_iters;
    info->eps = hs.eps;
    info->err2 = hs.err2;
    info->mu = hs.mu;
    info->mu0 = hs.mu0;
    info->cg_trials = fl[11];
    info->cg_iters = fl[12];
    info->t_done = 0.0;
  }
  if (hs.reason == DGN_STOP_NONFINITE) return set_err(ctx, DGN_ENONFINITE, "non-finite error or step");
  return DGN_OK;
}


dgn_status cp_als(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, void* const* A, int32_t sweeps,
                  const dgn_opts* opts, double* err2_out, void* stream) {
  if (!ctx) return DGN_EINVAL;
  if (!A) return set_err(ctx, DGN_EINVAL, "factor pointer array is NULL");
  if (sweeps < 0) return set_err(ctx, DGN_EINVAL, "sweeps must be >= 0");
  dgn_opts o;
  dgn_opts_default(&o);
  if (opts) o = *opts;
  Work w{};
  dgn_status rc = prepare(ctx, Y, R, false, w);
  if (rc != DGN_OK) return rc;
  for (int n = 0; n < w.s.N; ++n)
    if (!A[n]) return set_err(ctx, DGN_EINVAL, "NULL factor pointer");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  const Shape& s = w.s;
  // the updates use the plain MTTKRP; the error after the last sweep is taken
  // from the residual pass for FP64 and complex tensors (cancellation-free, and
  // the form the complex fit uses), otherwise from ||Y||^2 - 2 <Y, Y_hat> + ||Y_hat||^2
  const PassSel plain = pass_tensor(w, Y, o, false);
  const bool resid_err = (w.ymaster == YType::F64) || w.cs == 2;
  const long long J = [&] { long long j = 1; for (int n = 0; n < s.N; ++n) j *= s.I[n]; return j; }();
  double* ynp = w.scr + 1028;
  double* e2 = w.scr + 1024;
  double* out = w.scr + 1026;
  HIPCHK(hipMemsetAsync(w.flags, 0, 64 * sizeof(int), st), "memset");
  HIPCHK(copy_factors_in(w, A, w.A, st), "copy factors");
  HIPCHK(enqueue_als(w, plain, sweeps, w.flags, st), "als");
  HIPCHK(run_gram(w, w.A, w.sb.C, nullptr, st), "gram");
  if (resid_err) {
    HIPCHK(run_pass(w, PassSel{Y->data, w.ymaster}, w.A, true, w.M, e2, nullptr, st), "pass");
  } else {
    HIPCHK(run_norm2(plain, J, w.scr, ynp, st), "norm");
    HIPCHK(run_pass(w, plain, w.A, false, w.M, nullptr, nullptr, st), "pass");
  }
  HIPCHK(launch_err2(s, w.A, w.M, w.sb.C, resid_err, e2, ynp, out, st), "err2");
  HIPCHK(copy_factors_out(w, w.A, A, st), "copy out");
  double host = 0.0;
  int flags[1] = {0};
  HIPCHK(hipMemcpyAsync(&host, out, sizeof host, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st), "copy");
  HIPCHK(hipStreamSynchronize(st), "sync");
  if (err2_out) *err2_out = host;
  if (flags[0]) return set_err(ctx, DGN_ESINGULAR, "a Gamma^(n) of the ALS update is not positive definite");
  if (!isfinite(host)) return set_err(ctx, DGN_ENONFINITE, "non-finite error after the ALS sweeps");
  return DGN_OK;
}

// ---- mode-n singular vectors (SVD initialisation) ---------------------------

namespace {

constexpr int kMaxSvdBlock = 80;

struct SvdWork {
  SvdModes m;
  double* part;
  double* sigma;
  int* bad;
  // complex tensors: the problem in m is the real embedding (doubled sizes)
  bool cplx = false;
  double* Gp = nullptr;   // real Gram of the interleaved rows, (2 I_n)^2 for the largest mode
  double* svr = nullptr;  // N x 2R singular values of the embedding
};

// Validates the tensor for the SVD calls (no rank check beyond 1 <= R) and
// fills s / yt.
dgn_status check_svd_tensor(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, Shape* s, YType* yt) {
  const int32_t rr = (R >= 1 && R <= kMaxRankC) ? R : 1;
  return check_shape(ctx, Y, rr, s, yt);
}

// Complex tensors run the real pipeline on the embeddings [[G_re, -G_im],
// [G_im, G_re]] of their Hermitian Grams: sizes, block and rank doubled.
void carve_svd(Arena& ar, const Shape& s, int R, int b, bool cplx, SvdWork& w) {
  const int f = cplx ? 2 : 1;
  SvdModes& m = w.m;
  w.cplx = cplx;
  m.N = s.N;
  m.b = f * b;
  m.bp = (m.b + 15) / 16 * 16;
  m.R = f * R;
  m.blk0[0] = 0;
  size_t gp = 0;
  for (int n = 0; n < s.N; ++n) {
    m.I[n] = f * s.I[n];
    m.Ip[n] = (m.I[n] + 63) / 64 * 64;
    m.G[n] = ar.take<double>((size_t)m.Ip[n] * m.Ip[n]);
    m.Q[n] = ar.take<double>((size_t)m.Ip[n] * m.bp);
    m.Z[n] = ar.take<double>((size_t)m.Ip[n] * m.bp);
    m.A[n] = cplx ? ar.take<double>((size_t)m.I[n] * m.R) : nullptr;
    m.blk0[n + 1] = m.blk0[n] + (m.Ip[n] / 64) * (m.bp / 16);
    const size_t g2 = (size_t)m.I[n] * m.I[n];
    if (g2 > gp) gp = g2;
  }
  w.part = ar.take<double>(cplx ? gram_part_doubles_c(s) : gram_part_doubles(s));
  w.sigma = ar.take<double>(kMaxOrder);
  w.bad = ar.take<int>(64);
  if (cplx) {
    w.Gp = ar.take<double>(gp);
    w.svr = ar.take<double>((size_t)s.N * m.R);
  }
}

dgn_status check_svd_args(dgn_ctx* ctx, const Shape& s, bool cplx, int32_t R, int32_t block, int32_t iters) {
  int mn = s.I[0];
  for (int n = 1; n < s.N; ++n) mn = s.I[n] < mn ? s.I[n] : mn;
  const int rmax = cplx ? kMaxRankC : DGN_MAX_RANK;
  const int bmax = cplx ? kMaxSvdBlock / 2 : kMaxSvdBlock;
  if (R < 1 || R > rmax) return set_err(ctx, DGN_EINVAL, cplx ? "complex tensors need rank in [1, 32]" : "rank must be in [1, 64]");
  if (R > mn) return set_err(ctx, DGN_EINVAL, "the SVD initialisation needs R <= every I_n");
  if (block < R || block > mn || block > bmax)
    return set_err(ctx, DGN_EINVAL, "block must satisfy R <= block <= min(min_n I_n, 80; 40 for complex tensors)");
  if (iters < 0) return set_err(ctx, DGN_EINVAL, "iters must be >= 0");
  return DGN_OK;
}

}  // namespace

dgn_status dgn_workspace_size_svd(const dgn_tensor* Y, int32_t R, int32_t block, size_t* bytes) {
  if (!bytes) return DGN_EINVAL;
  Shape s{};
  YType yt;
  dgn_status st = check_svd_tensor(nullptr, Y, R, &s, &yt);
  if (st != DGN_OK) return st;
  if ((st = check_svd_args(nullptr, s, is_complex(yt), R, block, 0)) != DGN_OK) return st;
  Arena ar{nullptr, (size_t)-1};
  SvdWork w{};
  carve_svd(ar, s, R, block, is_complex(yt), w);
  *bytes = ar.used;
  return DGN_OK;
}

dgn_status dgn_mode_gram(dgn_ctx* ctx, const dgn_tensor* Y, int32_t n, double* G, void* stream) {
  if (!ctx) return DGN_EINVAL;
  Shape s{};
  YType yt;
  dgn_status st = check_svd_tensor(ctx, Y, 1, &s, &yt);
  if (st != DGN_OK) return st;
  if (n < 0 || n >= s.N) return set_err(ctx, DGN_EINVAL, "mode index out of range");
  if (!G) return set_err(ctx, DGN_EINVAL, "output pointer is NULL");
  const bool cplx = is_complex(yt);
  Arena ar{ctx->ws, ctx->ws_size};
  double* part = ar.take<double>(cplx ? gram_part_doubles_c(s) : gram_part_doubles(s));
  double* Gp = cplx ? ar.take<double>((size_t)4 * s.I[n] * s.I[n]) : nullptr;
  if (ar.fail)
    return set_err(ctx, DGN_ENOMEM, "workspace budget too small: need " + std::to_string(ar.used) + " bytes");
  hipStream_t hs = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  if (cplx)
    HIPCHK(launch_mode_gram_c(s, n, Y->data, yt, part, Gp, nullptr, 0, G, hs), "mode gram");
  else
    HIPCHK(launch_mode_gram(s, n, Y->data, yt, part, G, s.I[n], s.I[n], hs), "mode gram");
  return DGN_OK;
}

dgn_status cp_svd_init(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, int32_t block, const double* omega,
                       int32_t iters, void* const* A, double* sv, void* stream) {
  if (!ctx) return DGN_EINVAL;
  Shape s{};
  YType yt;
  dgn_status st = check_svd_tensor(ctx, Y, R, &s, &yt);
  if (st != DGN_OK) return st;
  const bool cplx = is_complex(yt);
  if ((st = check_svd_args(ctx, s, cplx, R, block, iters)) != DGN_OK) return st;
  if (!omega) return set_err(ctx, DGN_EINVAL, "start block pointer is NULL");
  if (!A) return set_err(ctx, DGN_EINVAL, "factor pointer array is NULL");
  for (int n = 0; n < s.N; ++n)
    if (!A[n]) return set_err(ctx, DGN_EINVAL, "NULL factor pointer");
  Arena ar{ctx->ws, ctx->ws_size};
  SvdWork w{};
  carve_svd(ar, s, R, block, cplx, w);
  if (ar.fail)
    return set_err(ctx, DGN_ENOMEM, "workspace budget too small: need " + std::to_string(ar.used) + " bytes");
  hipStream_t hs = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  HIPCHK(hipMemsetAsync(w.bad, 0, sizeof(int), hs), "memset");
  if (cplx) {
    CxFactors out{};
    for (int n = 0; n < s.N; ++n) out.A[n] = (double*)A[n];
    HIPCHK(launch_svd_init_c(s, Y->data, yt, w.m, out, w.Gp, omega, iters, w.part, w.sigma, w.svr, sv, w.bad, hs),
           "svd init");
  } else {
    for (int n = 0; n < s.N; ++n) w.m.A[n] = (double*)A[n];
    HIPCHK(launch_svd_init(s, Y->data, yt, w.m, omega, iters, w.part, w.sigma, sv, w.bad, hs), "svd init");
  }
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, w.bad, sizeof bad, hipMemcpyDeviceToHost, hs), "copy");
  HIPCHK(hipStreamSynchronize(hs), "sync");
  if (bad) return set_err(ctx, DGN_ESINGULAR, "the orthonormalisation of the subspace iteration broke down");
  return DGN_OK;
}

dgn_status cp_fit_batched(dgn_ctx* ctx, int32_t B, const dgn_batch_fit* fits, double tol,
                          int32_t max_iters, const dgn_opts* opts, dgn_fit_info* infos,
                          void* stream) {
  if (!ctx) return DGN_EINVAL;
  if (B < 0 || (B > 0 && !fits)) return set_err(ctx, DGN_EINVAL, "bad batch size or NULL fits");
  if (opts && opts->als_sweeps != 0)
    return set_err(ctx, DGN_EINVAL, "cp_fit_batched has no ALS warm-up (als_sweeps must be 0)");
  if (max_iters < 0 || !(tol >= 0.0)) return set_err(ctx, DGN_EINVAL, "need max_iters >= 0 and tol >= 0");
  if (B == 0) return DGN_OK;
  dgn_opts o;
  dgn_opts_default(&o);
  if (opts) o = *opts;
  if (o.poll_every < 1) o.poll_every = 1;
  if (o.mu_rule != DGN_MU_PAPER && o.mu_rule != DGN_MU_NIELSEN) return set_err(ctx, DGN_EINVAL, "bad mu_rule option");
  // validate and size the workspace
  size_t need = 0;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  std::vector<BFit> hf(B);
  for (int b = 0; b < B; ++b) {
    const dgn_batch_fit& f = fits[b];
    if (!f.Y.data || (f.Y.dtype != DGN_F32 && f.Y.dtype != DGN_F64) ||
        !batched_supported(f.Y.order, f.Y.dims, f.R) || !f.A[0] || !f.A[1] || !f.A[2] || !isfinite(f.mu0))
      return set_err(ctx, DGN_EINVAL, "batch fit " + std::to_string(b) +
                                          ": need order 3, F32/F64 data, I_n <= 64, 1 <= R <= 8, non-NULL factors");
    need += batched_ws_fit(f.Y.dims, f.R);
  }
  need += batched_ws_call(B);
  if (o.batched_launch < DGN_BATCH_AUTO || o.batched_launch > DGN_BATCH_PERSISTENT)
    return set_err(ctx, DGN_EINVAL, "bad batched_launch option");
  if (need > ctx->ws_size)
    return set_err(ctx, DGN_ENOMEM, "workspace budget too small for the batch: need " + std::to_string(need));
  hipStream_t cs = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  if (!ctx->own) HIPCHK(hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking), "hipStreamCreate");
  hipStream_t st = ctx->own;
  char* base = ctx->ws;
  size_t used = 0;
  auto take = [&](size_t bytes) { char* p = base + used; used += al(bytes); return p; };
  BFit* dfits = reinterpret_cast<BFit*>(take(sizeof(BFit) * (size_t)B));
  int* nstopped = reinterpret_cast<int*>(take(sizeof(int) * 64));  // [0] stopped fits, [1] persistent queue
  int* dorder = reinterpret_cast<int*>(take(sizeof(int) * (size_t)B));
  std::vector<FitState*> states(B);
  for (int b = 0; b < B; ++b) {
    const dgn_batch_fit& f = fits[b];
    BFit& h = hf[b];
    h.Y = f.Y.data;
    h.dtype = (f.Y.dtype == DGN_F64) ? 0 : 1;
    for (int n = 0; n < 3; ++n) h.I[n] = (int)f.Y.dims[n];
    h.R = f.R;
    h.mu0 = f.mu0;
    const size_t TR = (size_t)(h.I[0] + h.I[1] + h.I[2]) * f.R;
    double* w = reinterpret_cast<double*>(take(batched_fit_doubles(h.I, f.R) * sizeof(double)));
    h.A = w;
    h.Ac = w + TR;
    h.M = w + 2 * TR;
    h.Mc = w + 3 * TR;
    h.G = w + 4 * TR;
    h.P = w + 5 * TR;
    h.C = w + 6 * TR;
    h.Cc = h.C + 3 * 64;
    for (int n = 0; n < 3; ++n) h.Ain[n] = static_cast<double*>(f.A[n]);
    h.st = reinterpret_cast<FitState*>(take(sizeof(FitState)));
    states[b] = h.st;
  }
  BatchCfg cfg{tol, o.tau, o.resid_switch, max_iters, o.normalize, o.mu_rule, nstopped};
  // order the private stream after the caller's work
  hipEvent_t ev_in, ev_out;
  HIPCHK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming), "event");
  HIPCHK(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming), "event");
  HIPCHK(hipEventRecord(ev_in, cs), "event");
  HIPCHK(hipStreamWaitEvent(st, ev_in, 0), "event");
  HIPCHK(hipMemcpyAsync(dfits, hf.data(), sizeof(BFit) * (size_t)B, hipMemcpyHostToDevice, st), "copy fits");
  HIPCHK(hipMemsetAsync(nstopped, 0, sizeof(int), st), "memset");
  // Fits in decreasing order of their per-trial tensor work (largest first), the
  // queue order of the persistent launch.
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const double wx = (double)hf[x].I[0] * hf[x].I[1] * hf[x].I[2] * hf[x].R;
    const double wy = (double)hf[y].I[0] * hf[y].I[1] * hf[y].I[2] * hf[y].R;
    return wx > wy;
  });
  HIPCHK(hipMemcpyAsync(dorder, order.data(), sizeof(int) * (size_t)B, hipMemcpyHostToDevice, st), "copy order");
  int ncu = 0;
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device), "device attribute");
  const int pblocks = ncu > 0 ? ncu : 256;  // the trial kernel's LDS allows one block per CU
  int launch = o.batched_launch;
  if (launch == DGN_BATCH_AUTO) launch = DGN_BATCH_GRAPH;
  if (o.batched_launch == DGN_BATCH_AUTO && max_iters > 0) {
    int imax = 1, rmax = 1;
    for (int b = 0; b < B; ++b) {
      rmax = std::max(rmax, hf[b].R);
      for (int n = 0; n < 3; ++n) imax = std::max(imax, hf[b].I[n]);
    }
    const std::pair<int, int> key((imax + 15) / 16, rmax);
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        launch = it->second.launch;
        have = true;
      }
    }
    if (!have) {
      // Time both shapes on (up to) 256 fits spread over the batch's order, from
      // their initial states through a few trials; the caller's factors are not
      // touched, and every state is initialised again by the run below.
      const int ns = std::min(B, 256), nt = std::min(max_iters, 4);
      std::vector<BFit> sample(ns);
      for (int k = 0; k < ns; ++k) sample[k] = hf[order[(long long)k * B / ns]];
      std::vector<int> sorder(ns);
      for (int k = 0; k < ns; ++k) sorder[k] = k;
      HIPCHK(hipMemcpyAsync(dfits, sample.data(), sizeof(BFit) * (size_t)ns, hipMemcpyHostToDevice, st), "copy sample");
      HIPCHK(hipMemcpyAsync(dorder, sorder.data(), sizeof(int) * (size_t)ns, hipMemcpyHostToDevice, st), "copy order");
      hipEvent_t t0, t1, t2;
      HIPCHK(hipEventCreate(&t0), "event");
      HIPCHK(hipEventCreate(&t1), "event");
      HIPCHK(hipEventCreate(&t2), "event");
      HIPCHK(hipEventRecord(t0, st), "event");
      HIPCHK(launch_batched_init(dfits, ns, cfg, st), "tune init");
      for (int k = 0; k < nt; ++k) HIPCHK(launch_batched_trial(dfits, ns, cfg, st), "tune trial");
      HIPCHK(hipEventRecord(t1, st), "event");
      HIPCHK(launch_batched_persistent(dfits, ns, dorder, nstopped + 1, cfg, pblocks, nt, false, st), "tune persistent");
      HIPCHK(hipEventRecord(t2, st), "event");
      HIPCHK(hipEventSynchronize(t2), "sync");
      float ms_g = 0.f, ms_p = 0.f;
      HIPCHK(hipEventElapsedTime(&ms_g, t0, t1), "elapsed");
      HIPCHK(hipEventElapsedTime(&ms_p, t1, t2), "elapsed");
      hipEventDestroy(t0);
      hipEventDestroy(t1);
      hipEventDestroy(t2);
      BatchTune bt;
      bt.launch = ms_p < ms_g ? DGN_BATCH_PERSISTENT : DGN_BATCH_GRAPH;
      bt.us_graph = 1e3 * ms_g / ((double)ns * nt);
      bt.us_persistent = 1e3 * ms_p / ((double)ns * nt);
      bt.sample_fits = ns;
      bt.sample_trials = nt;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = bt;
      }
      launch = bt.launch;
      HIPCHK(hipMemcpyAsync(dfits, hf.data(), sizeof(BFit) * (size_t)B, hipMemcpyHostToDevice, st), "copy fits");
      HIPCHK(hipMemcpyAsync(dorder, order.data(), sizeof(int) * (size_t)B, hipMemcpyHostToDevice, st), "copy order");
      HIPCHK(hipMemsetAsync(nstopped, 0, sizeof(int), st), "memset");
    }
  }
  ctx->batch_launch = launch;
  if (launch == DGN_BATCH_PERSISTENT) {
    HIPCHK(launch_batched_persistent(dfits, B, dorder, nstopped + 1, cfg, pblocks, max_iters, true, st), "persistent");
  } else {
  HIPCHK(launch_batched_init(dfits, B, cfg, st), "batched init");
  const int per = o.poll_every < max_iters ? o.poll_every : (max_iters > 0 ? max_iters : 1);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (o.graph && max_iters > 0) {
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "capture");
    for (int k = 0; k < per; ++k) launch_batched_trial(dfits, B, cfg, st);
    HIPCHK(hipStreamEndCapture(st, &graph), "capture end");
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
  }
  int done = 0, host_stopped = 0;
  while (done < max_iters) {
    if (exec) {
      HIPCHK(hipGraphLaunch(exec, st), "graph launch");
    } else {
      for (int k = 0; k < per; ++k) HIPCHK(launch_batched_trial(dfits, B, cfg, st), "batched trial");
    }
    done += per;
    HIPCHK(hipMemcpyAsync(&host_stopped, nstopped, sizeof(int), hipMemcpyDeviceToHost, st), "poll");
    HIPCHK(hipStreamSynchronize(st), "sync");
    if (host_stopped >= B) break;
  }
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  HIPCHK(launch_batched_final(dfits, B, st), "batched final");
  }
  std::vector<FitState> hs(B);
  for (int b = 0; b < B; ++b)
    HIPCHK(hipMemcpyAsync(&hs[b], states[b], sizeof(FitState), hipMemcpyDeviceToHost, st), "state");
  HIPCHK(hipEventRecord(ev_out, st), "event");
  HIPCHK(hipStreamWaitEvent(cs, ev_out, 0), "event");
  HIPCHK(hipStreamSynchronize(st), "sync");
  hipEventDestroy(ev_in);
  hipEventDestroy(ev_out);
  int nonfinite = 0;
  int clk_khz = 0;
  if (hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess) clk_khz = 0;
  long long tstart = hs.empty() ? 0 : hs[0].t0_ticks;
  for (int b = 0; b < B; ++b) tstart = std::min(tstart, hs[b].t0_ticks);
  for (int b = 0; b < B; ++b) {
    if (infos) {
      infos[b].t_done = clk_khz > 0 ? (double)(hs[b].t1_ticks - tstart) / (1e3 * clk_khz) : 0.0;
      infos[b].iters = hs[b].iters;
      infos[b].accepted = hs[b].accepted;
      infos[b].reason = hs[b].reason;
      infos[b].resid_iters = hs[b].resid_iters;
      infos[b].eps = hs[b].eps;
      infos[b].err2 = hs[b].err2;
      infos[b].mu = hs[b].mu;
      infos[b].mu0 = hs[b].mu0;
      infos[b].cg_trials = 0;
      infos[b].cg_iters = 0;
    }
    nonfinite += hs[b].reason == DGN_STOP_NONFINITE;
  }
  if (nonfinite) return set_err(ctx, DGN_ENONFINITE, std::to_string(nonfinite) + " fit(s) stopped on a non-finite step");
  return DGN_OK;
}

dgn_status dgn_batched_tuning(dgn_batch_tune_entry* out, int32_t max, int32_t* n) {
  if (!n || max < 0 || (max > 0 && !out)) return DGN_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int k = 0;
  for (const auto& kv : g_tune) {
    if (k >= max) break;
    out[k].imax_bucket = kv.first.first * 16;
    out[k].rmax = kv.first.second;
    out[k].launch = kv.second.launch;
    out[k].us_per_trial_graph = kv.second.us_graph;
    out[k].us_per_trial_persistent = kv.second.us_persistent;
    out[k].sample_fits = kv.second.sample_fits;
    out[k].sample_trials = kv.second.sample_trials;
    ++k;
  }
  *n = k;
  return DGN_OK;
}

int32_t dgn_batched_last_launch(const dgn_ctx* ctx) { return ctx ? ctx->batch_launch : -1; }

}  // extern "C"
