/*
 * dgn.h -- C ABI of the MI355X (gfx950) fast damped Gauss-Newton library for
 * CANDECOMP/PARAFAC (Phan, Tichavsky, Cichocki, "Low complexity damped
 * Gauss-Newton algorithms for CANDECOMP/PARAFAC").
 *
 * Conventions shared by every call
 * --------------------------------
 * - A tensor Y of order N (3 <= N <= DGN_MAX_ORDER) with sizes I_1..I_N is a
 *   dense device buffer holding vec(Y) with the first index fastest
 *   (column-major), the vectorisation of Section 2.  Y_(n) is never formed.
 * - A factor A^(n) is a device buffer of I_n x R doubles (complex doubles
 *   for complex tensors), column-major, leading dimension I_n.  Factors are
 *   passed as a host array of N device pointers.
 * - All device pointers are caller-owned.  The library never frees them and
 *   never keeps them after a call returns.
 * - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   Work is enqueued on that stream.  Calls that return host results
 *   (dgn_step_info, dgn_fit_info, inner products) synchronise the stream
 *   before returning.
 * - A context is bound to one device and is not thread-safe: one context per
 *   host thread / stream.
 * - Every call returns a dgn_status; on failure dgn_last_error() gives a
 *   readable message.  Shapes are validated before any work is enqueued:
 *   order in [3, DGN_MAX_ORDER], every I_n >= 1, 1 <= R <= DGN_MAX_RANK
 *   (R <= DGN_MAX_RANK_COMPLEX for C64/C128 tensors), mu > 0 (H = J^T J is
 *   singular, so mu = 0 is rejected), non-NULL pointers.
 *
 * Arithmetic
 * ----------
 * The tensor pass (MTTKRP and the residual) runs in the tensor's dtype:
 * F64 -> FP64; F32 -> FP32 MFMA with FP32 accumulation; BF16 -> BF16 MFMA
 * with FP32 accumulation; C128 and C64 -> FP64 complex (C64 entries are read
 * as complex64 and widened).  Partial sums are reduced in FP64.  Everything
 * after the tensor pass (Gram and Hadamard products, the damped inverses, the
 * NR^2 system and the factor update) is FP64 (complex FP64).
 *
 * Complex tensors (Section 5): factors are complex128, stored as interleaved
 * (re, im) pairs in the same column-major I_n x R layout.  The step always
 * uses the residual form of the tensor pass, and the Hermitian positive
 * definite NR^2 system is solved through its real symmetric embedding
 * [[Re S, -Im S], [Im S, Re S]] by the same tiled Cholesky as the real case.
 */
#ifndef DGN_H
#define DGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGN_MAX_ORDER 8
#define DGN_MAX_RANK 64
#define DGN_MAX_RANK_COMPLEX 32

typedef enum dgn_status {
  DGN_OK = 0,
  DGN_EINVAL = -1,     /* bad shape, rank, dtype, mu or NULL pointer */
  DGN_ENOMEM = -2,     /* workspace budget of the context too small */
  DGN_ESINGULAR = -3,  /* non-positive pivot in (Gamma^(n) + mu I) or the NR^2 system */
  DGN_ENONFINITE = -4, /* NaN/Inf in the tensor pass or the step */
  DGN_EHIP = -5,       /* a HIP runtime call failed */
  DGN_EBUSY = -6       /* request over the memory budget (serving) */
} dgn_status;

typedef enum dgn_dtype {
  DGN_F64 = 0,
  DGN_F32 = 1,
  DGN_BF16 = 2,
  DGN_C64 = 3,
  DGN_C128 = 4
} dgn_dtype;

typedef enum dgn_normalize {
  DGN_NORM_BALANCED = 0,        /* equal column norms across modes (Algorithm 1, normalisation step) */
  DGN_NORM_UNIT_EXCEPT_LAST = 1,/* unit columns in modes 1..N-1 (Section 2) */
  DGN_NORM_NONE = 2
} dgn_normalize;

typedef enum dgn_stop {
  DGN_STOP_TOL = 0,       /* |eps_prev - eps| < tol on an accepted trial */
  DGN_STOP_MAX_IT = 1,    /* max_iters trials done */
  DGN_STOP_MU = 2,        /* mu > 1e30 (Section 4.5) */
  DGN_STOP_NONFINITE = 3  /* non-finite error or step */
} dgn_stop;

/* Dense tensor descriptor.  dims[k] for k >= order are ignored.  `data` is a
 * device pointer to prod(dims) elements of `dtype`, first index fastest. */
typedef struct dgn_tensor {
  int32_t order;
  int64_t dims[DGN_MAX_ORDER];
  int32_t dtype; /* dgn_dtype */
  const void* data;
} dgn_tensor;

/* Options.  dgn_opts_default() fills the defaults; NULL opts means defaults. */
typedef struct dgn_opts {
  int32_t normalize;    /* dgn_normalize, default BALANCED */
  double tau;           /* mu0 = tau * max_n max diag Gamma^(n) when mu0 <= 0 (eq. mu0); default 1e-3 */
  /* Real F32/BF16 tensors: the gradient is first taken from the plain
   * MTTKRP, and the error from ||Y||^2 - 2<Y,Y_hat> + ||Y_hat||^2.  Once an
   * accepted trial changes the relative error eps by less than resid_switch
   * the fit switches to the residual-corrected pass: E = Y - Y_hat is formed
   * in FP32 inside the pass, the gradient is MTTKRP(E) and the error is
   * sum(E^2).  0 never switches, a negative value starts residual-corrected.
   * F64/C128 tensors always use the residual form.  Default 1e-3: a BF16
   * tensor carries about 2^-9 relative rounding per entry, so changes of eps
   * below that level have to be judged from the exact residual. */
  double resid_switch;
  /* Optional BF16 copy of Y (same dims, device) used by the plain passes of
   * an F32 tensor before the switch.  NULL: the F32 tensor is used. */
  const void* y_bf16;
  int32_t poll_every;   /* cp_fit checks its stop flag every this many trials; default 8 */
  int32_t timing;       /* nonzero: cp_fit records per-phase HIP events (dgn_last_phase_times) */
  int32_t graph;        /* cp_fit_batched: nonzero (default) replays poll_every trials from one
                           captured hipGraph; zero launches them one by one */
  int32_t als_sweeps;   /* cp_fit and the server: ALS sweeps (as cp_als) on the starting factors
                           before the first trial; default 0.  cp_fit_batched rejects a nonzero
                           value with DGN_EINVAL */
  /* dgn_step and cp_fit, N <= 4 and R <= 32 (complex tensors: R <= 16): DGN_SOLVER_AUTO
   * first solves the NR^2 system by conjugate gradients on its structured SPD
   * form (Section 4.3: Kronecker and permuted-diagonal products, the matrix is
   * never formed; Hermitian for complex tensors, Section 5) and runs the direct
   * tiled Cholesky only when CG has not
   * reached ||r|| <= cg_tol ||z|| within cg_max_iters iterations, or earlier
   * when it cannot: every 10 iterations from the 20th the mean reduction of
   * ||r||^2 per iteration so far is extrapolated, and an attempt whose goal
   * lies beyond 2 cg_max_iters at that rate is abandoned (so a hopeless
   * attempt costs about 20 iterations); inside cp_fit
   * the first such failure leaves CG out for the rest of the fit.  The step
   * then differs from the direct one by the CG tolerance (amplified by the
   * condition number of the system).  Default DGN_SOLVER_DIRECT. */
  int32_t solver;
  int32_t cg_max_iters; /* default 100 */
  double cg_tol;        /* default 1e-10 */
  /* cp_fit, cp_fit_batched and the server: growth of mu on a rejected trial
   * (Section 4.5).  DGN_MU_PAPER (default): mu <- 2 mu, as the section prints
   * it.  DGN_MU_NIELSEN: the rule of the damping reference the section cites,
   * mu <- mu nu and nu <- 2 nu on a rejection, nu reset to 2 on an acceptance,
   * so that a run of rejections grows mu ever faster.  The decrease on an
   * accepted trial is the same under both. */
  int32_t mu_rule;
  /* cp_fit_batched: how the trials are launched.  DGN_BATCH_GRAPH: one block per
   * fit per trial, trials replayed from a captured hipGraph (or launched one by
   * one with graph = 0).  DGN_BATCH_PERSISTENT: one block per CU, each taking the
   * next fit from a queue (largest first) and running it to its stop.
   * DGN_BATCH_AUTO (default): the shape the library's tuner measured faster for
   * batches of this largest mode size (buckets of 16) and largest rank; the first
   * call with a new key times both shapes on up to 256 of its fits for a few
   * trials (dgn_batched_tuning lists the table).  Every shape gives each fit the
   * same result. */
  int32_t batched_launch;
  /* dgn_server: route requests within the batched shapes (order 3, F32/F64
   * data, I_n <= 64, R <= 8) to a batch lane that runs every such request
   * pending at the time, grouped by (tol, max_iters), in one cp_fit_batched
   * call with the persistent launch; the next group forms while it runs.
   * Default 1; 0 runs every request in a slot as cp_fit. */
  int32_t serve_batch;
} dgn_opts;

typedef enum dgn_solver { DGN_SOLVER_DIRECT = 0, DGN_SOLVER_AUTO = 1 } dgn_solver;
typedef enum dgn_mu_rule { DGN_MU_PAPER = 0, DGN_MU_NIELSEN = 1 } dgn_mu_rule;
typedef enum dgn_batch_launch { DGN_BATCH_AUTO = 0, DGN_BATCH_GRAPH = 1, DGN_BATCH_PERSISTENT = 2 } dgn_batch_launch;

/* Result of one trial step (dgn_step). */
typedef struct dgn_step_info {
  double err2_old;  /* ||Y - Y_hat(A_in)||^2 */
  double err2_new;  /* ||Y - Y_hat(A_out)||^2 */
  double rho;       /* (err2_old - err2_new) / denom  (gain ratio, Section 4.5) */
  double denom;     /* Re(da^H (g + mu da)) */
  double gnorm;     /* ||g||, g = J^H vec(Y - Y_hat) */
  double mnorm;     /* ||[M_n]||, all-mode MTTKRP norm (plain form) or ||[M_n - A_n Gamma_n]|| is g */
  double danorm;    /* ||da|| */
  int32_t cg_iters; /* DGN_SOLVER_AUTO: CG iterations of a converged CG solve, -1 when the direct solve ran */
  int32_t cg_attempt_iters; /* DGN_SOLVER_AUTO: iterations of the CG attempt, converged or abandoned
                               (the direct solve then ran); -1 when CG was not tried */
} dgn_step_info;

/* Result of a fit (cp_fit). */
typedef struct dgn_fit_info {
  int32_t iters;        /* trials done (accepted + rejected) */
  int32_t accepted;     /* accepted trials */
  int32_t reason;       /* dgn_stop */
  int32_t resid_iters;  /* trials taken with the residual-corrected pass */
  double eps;           /* final ||Y - Y_hat|| / ||Y|| */
  double err2;          /* final ||Y - Y_hat||^2 */
  double mu;            /* final damping */
  double mu0;           /* initial damping actually used */
  int32_t cg_trials;    /* DGN_SOLVER_AUTO: trials whose NR^2 system CG solved (else 0) */
  int32_t cg_iters;     /* their CG iterations, summed */
  double t_done;        /* cp_fit_batched: seconds from the first fit's initial state to this fit's
                           stop (device clock), the fit's latency inside the batch; 0 elsewhere */
} dgn_fit_info;

typedef struct dgn_ctx dgn_ctx;

/* Fill *opts with the defaults listed in dgn_opts. */
void dgn_opts_default(dgn_opts* opts);

/* Create a context on `device` owning a device workspace of ws_budget_bytes
 * (allocated once here; 0 picks 1 GiB).  Calls needing more return
 * DGN_ENOMEM; dgn_workspace_size() gives the requirement. */
dgn_status dgn_create(dgn_ctx** out, int32_t device, size_t ws_budget_bytes);
dgn_status dgn_destroy(dgn_ctx* ctx);
/* Message of the last failure on this context ("" if none).  Owned by ctx.
 * ctx == NULL: the last failure of dgn_step_noalloc on the calling thread. */
const char* dgn_last_error(const dgn_ctx* ctx);

/* Workspace bytes dgn_step / cp_fit / dgn_mttkrp need for this shape. */
dgn_status dgn_workspace_size(const dgn_tensor* Y, int32_t R, const dgn_opts* opts, size_t* bytes);

/* All-mode MTTKRP (Section 4.4, the O(NRJ) step; eq. ALS numerator):
 * M_n = Y_(n) (A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1)) for
 * every n, with conjugated factors for complex tensors (Theorem 5.4), in one
 * pass over Y.  A: N device pointers to I_n x R FP64 (C128) factors; the pass
 * casts them to the tensor's compute type.  M: N device pointers to I_n x R
 * FP64 (C128) outputs.  inner (host, may be NULL): <Y, Y_hat> = sum(A_1 * M_1);
 * for complex tensors Re sum(conj(A_1) * M_1) = Re sum(y conj(y_hat)).
 * Synchronises when inner != NULL. */
dgn_status dgn_mttkrp(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, const void* const* A,
                      void* const* M, double* inner, void* stream);

/* One trial damped Gauss-Newton step at damping mu (Theorem 4.1 with the
 * Jacobian-free products of Lemma 4.4 and the fLMa solve of Section 4.3):
 * A_out = A_in + da with da = (J^H J + mu I)^-1 J^H vec(Y - Y_hat(A_in)).
 * A_out may alias A_in.  No normalisation and no accept/reject: `info`
 * (host, may be NULL) reports the errors before and after and the gain ratio.
 * Synchronises the stream before returning. */
dgn_status dgn_step(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, const void* const* A_in,
                    void* const* A_out, double mu, const dgn_opts* opts, dgn_step_info* info,
                    void* stream);

/* dgn_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same step, arguments, outputs and errors as dgn_step, but with no context.
 * Its workspace is a fixed scratch array inside the library, one per GPU,
 * of dgn_noalloc_scratch_bytes() bytes (64 MiB), held by every GPU the library
 * runs on until the process ends; the call allocates nothing and frees
 * nothing.  The device is the calling thread's current device.  A shape whose
 * workspace (dgn_workspace_size) exceeds the array gives DGN_ENOMEM with a
 * message from dgn_last_error(NULL), which also holds the message of any other
 * failure of this call on this thread.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other host threads, or streams
 * that run concurrently) race and give wrong results; serialise them.  The
 * call clears the parts of the array that must start at zero.  Synchronises
 * the stream before returning. */
dgn_status dgn_step_noalloc(const dgn_tensor* Y, int32_t R, const void* const* A_in, void* const* A_out,
                            double mu, const dgn_opts* opts, dgn_step_info* info, void* stream);
/* Size in bytes of the scratch array of dgn_step_noalloc. */
size_t dgn_noalloc_scratch_bytes(void);

/* The damped system with any right-hand side: X = (J^T J + mu I)^-1 V, the
 * inverse of H_mu applied in the block form of Section 4.1 (the memory-saving
 * representation: the R x R inverses (Gamma^(n) + mu I)^-1 and the NR^2
 * system, never the RT x RT inverse), with J the Jacobian of the CP model at the
 * factors A (Lemma B.1) -- dgn_step is this call with V = the gradient.  order,
 * dims: the mode sizes; dtype: DGN_F64, or DGN_C128 for complex factors
 * (Section 5: (J^H J + mu I)^-1, factors and blocks interleaved complex128);
 * A: N device pointers to I_n x R factors; V, X: N device pointers to I_n x R
 * column-major blocks (the parameter vector in blocks, as the factors are; X
 * may not alias V).  mu > 0; opts->solver selects the direct or the iterative
 * NR^2 solve as for dgn_step (real factors).
 * Workspace as dgn_workspace_size for an F64 tensor of these sizes.
 * Synchronises the stream before returning. */
dgn_status dgn_hessian_solve(dgn_ctx* ctx, int32_t order, const int64_t* dims, int32_t R, int32_t dtype,
                             const void* const* A, const void* const* V, void* const* X, double mu,
                             const dgn_opts* opts, void* stream);

/* The plain damped Gauss-Newton step of Section 3 with the Hessian formed
 * explicitly: (J^T J + mu I) da = J^T vec(Y - Y_hat), J^T J of size RT x RT
 * with the block form of Appendix B (diagonal blocks Gamma^(n) (x) I, off-diagonal
 * entries A_n[i, c] A_m[j, r] Gamma^(n,m)[r, c]), factored by the same tiled FP64
 * Cholesky as the fast step.  The paper's dGN baseline, for cost and memory
 * comparisons with dgn_step (Section 6); same arguments, outputs and errors as
 * dgn_step, real tensors only (a complex dtype gives DGN_EINVAL).  Its workspace,
 * about (RT)^2 x 8 bytes, comes from dgn_workspace_size_explicit.  Synchronises
 * the stream before returning. */
dgn_status dgn_step_explicit(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, const void* const* A_in,
                             void* const* A_out, double mu, const dgn_opts* opts, dgn_step_info* info,
                             void* stream);

/* Workspace bytes dgn_step_explicit needs for this shape (real tensors). */
dgn_status dgn_workspace_size_explicit(const dgn_tensor* Y, int32_t R, size_t* bytes);

/* Algorithm 1 with the damping of Section 4.5, device-resident.  A: in the
 * starting factors, out the result (N device pointers, FP64 / C128).
 * mu0 > 0 is used as given, mu0 <= 0 takes tau * max diag Gamma^(n).
 * Each trial: step at mu; accept iff the residual decreases, then normalise
 * and mu <- mu max(1/3, 1 - (2 rho - 1)^3); else mu grows by opts->mu_rule
 * (default mu <- 2 mu).  A trial whose (Gamma^(n) + mu I) or NR^2 system
 * meets a non-positive pivot in FP64 is rejected the same way (the damping is
 * too small for the system to be positive definite in working precision), so
 * cp_fit does not return DGN_ESINGULAR for the trials themselves.  Stops on an
 * accepted trial with |eps_prev - eps| < tol, after max_iters trials, or at
 * mu > 1e30.  Synchronises the stream before returning. */
dgn_status cp_fit(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, void* const* A, double mu0,
                  double tol, int32_t max_iters, const dgn_opts* opts, dgn_fit_info* info,
                  void* stream);

/* ALS warm-up (eq. ALS, Section 2; the paper runs a few ALS iterations after
 * initialising the factors, Section 4.5).  `sweeps` sweeps of
 *   A^(n) <- Y_(n) (Khatri-Rao of A^(k), k != n) (Gamma^(n))^-1,  n = 1..N in turn,
 * each update using the factors already updated in the sweep, with
 * Gamma^(n) = Hadamard_{k != n} A^(k)T A^(k) inverted through its Cholesky
 * factor (the pseudo-inverse of eq. ALS equals the inverse when every factor has
 * full column rank).  Complex tensors (Section 5) use the MTTKRP on conjugated
 * factors and (Gamma^(n)T)^-1, with Gamma^(n) the Hadamard product of
 * A^(k)H A^(k) (the least-squares solution).  A: N device pointers to I_n x R
 * column-major factors, FP64 (C128 for complex tensors), in the start and out
 * the result (caller-owned; no normalisation).  err2 (host, may be NULL)
 * receives ||Y - Y_hat||^2 after the last sweep (from the residual for F64 and
 * complex tensors, else from ||Y||^2 - 2 <Y, Y_hat> + ||Y_hat||^2); sweeps = 0
 * only evaluates it.  A Gamma^(n) that is not positive definite gives DGN_ESINGULAR
 * (the factors are then not meaningful).  Each mode update runs one all-mode
 * tensor pass.  Synchronises the stream before returning. */
dgn_status cp_als(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, void* const* A, int32_t sweeps,
                  const dgn_opts* opts, double* err2, void* stream);

/* Mode-n Gram matrix G = Y_(n) Y_(n)^T (I_n x I_n, FP64, column-major,
 * leading dimension I_n, both triangles written), the matrix whose leading
 * eigenvectors are the mode-n singular vectors used to initialise the factors
 * (Section 4.5).  Entries are widened to FP64 and products summed in FP64.
 * Complex tensors (C64, C128; Section 5): the Hermitian G = Y_(n) Y_(n)^H as
 * interleaved complex128.  n outside [0, order) gives DGN_EINVAL.  G:
 * caller-owned device buffer.  Uses the context's workspace (about 64 MB at
 * most for the partial tiles, plus (2 I_n)^2 doubles for complex tensors);
 * enqueued on `stream` without a synchronisation. */
dgn_status dgn_mode_gram(dgn_ctx* ctx, const dgn_tensor* Y, int32_t n, double* G, void* stream);

/* SVD initialisation (Section 4.5, as the experiments of Section 6 start):
 * A^(n) = the R leading left singular vectors of Y_(n), for every n, columns in
 * decreasing order of singular value, each column signed so that its entry of
 * largest magnitude (the first such on ties) is positive.  Computed as the
 * leading eigenvectors of Y_(n) Y_(n)^T (dgn_mode_gram) by `iters` steps of
 * subspace iteration with a block of `block` columns (R <= block <= min(min_n
 * I_n, 80); block > R speeds convergence of the R-th vector to the rate
 * ((lambda_{block+1} + s) / (lambda_R + s))^iters, s = 1e-7 trace) and a final
 * Rayleigh-Ritz step.  omega: device, the random start blocks, sum_n I_n x
 * block doubles, mode n's I_n x block column-major block after those of modes
 * < n.  A: N device pointers to I_n x R FP64 outputs.  sv (device, may be
 * NULL): N x R doubles, sv[n R + r] = r-th singular value of Y_(n).  Needs
 * R <= every I_n (DGN_EINVAL otherwise).  Complex tensors (Section 5): omega
 * and the factors are interleaved complex128, the vectors are fixed up to a
 * unit complex factor, chosen so that each column's largest-magnitude entry is
 * real and positive; R <= 32 and block <= 40, as the iteration runs on the real
 * embedding [[Re G, -Im G], [Im G, Re G]] of the Hermitian Gram.  DGN_ESINGULAR if
 * the orthonormalisation breaks down (omega of deficient rank).  Workspace
 * from dgn_workspace_size_svd.  Synchronises the stream before returning. */
dgn_status cp_svd_init(dgn_ctx* ctx, const dgn_tensor* Y, int32_t R, int32_t block, const double* omega,
                       int32_t iters, void* const* A, double* sv, void* stream);

/* Workspace bytes cp_svd_init needs for this shape, rank and block. */
dgn_status dgn_workspace_size_svd(const dgn_tensor* Y, int32_t R, int32_t block, size_t* bytes);

/* One small fit of a batch: a 3-way tensor (F32 or F64, every I_n <= 64),
 * rank 1 <= R <= 8, the initial damping (> 0 used as given, <= 0 the tau
 * rule) and three device pointers to FP64 column-major I_n x R factors
 * (in: start, out: result).  The batch owns none of these buffers. */
typedef struct dgn_batch_fit {
  dgn_tensor Y;
  int32_t R;
  double mu0;
  void* A[3];
} dgn_batch_fit;

/* B independent fits, each run exactly as cp_fit runs it (Algorithm 1 with
 * the damping of Section 4.5, same stop rules, tol and max_iters shared),
 * all advanced together, launched as opts->batched_launch selects (one block
 * per fit per trial from a replayed hipGraph, or a persistent queue of fits).
 * Fits stop independently.  infos (host, B entries, may be NULL) receives
 * each fit's result.  The tensor pass reads FP32 data and accumulates in
 * FP64.  Returns DGN_EINVAL if a fit is outside the supported shapes (order
 * 3, I_n <= 64, R <= 8).  Synchronises the stream before returning. */
dgn_status cp_fit_batched(dgn_ctx* ctx, int32_t B, const dgn_batch_fit* fits, double tol,
                          int32_t max_iters, const dgn_opts* opts, dgn_fit_info* infos,
                          void* stream);

/* One entry of the batched tuner's table: batches whose largest mode size is at
 * most imax_bucket (a multiple of 16) and whose largest rank is rmax run with
 * `launch` (dgn_batch_launch); the measured microseconds per fit-trial of each
 * shape on the sample (sample_fits fits, sample_trials trials from their starts). */
typedef struct dgn_batch_tune_entry {
  int32_t imax_bucket, rmax, launch;
  double us_per_trial_graph, us_per_trial_persistent;
  int32_t sample_fits, sample_trials;
} dgn_batch_tune_entry;

/* Copy up to max entries of the process-wide tuning table into out; *n receives
 * the count. */
dgn_status dgn_batched_tuning(dgn_batch_tune_entry* out, int32_t max, int32_t* n);
/* The launch shape (dgn_batch_launch) the last cp_fit_batched call on ctx used; -1 for NULL. */
int32_t dgn_batched_last_launch(const dgn_ctx* ctx);

/* ---- Serving: a request loop over cp_fit ------------------------------------
 * A server owns one device arena of budget_bytes.  Requests are admitted in
 * arrival order when a slot is free and their workspace (dgn_workspace_size)
 * fits in the free part of the arena; admitted requests run concurrently,
 * each on its own stream, so their kernels overlap on the device.  Requests
 * within the batched shapes go to the batch lane instead (opts->serve_batch):
 * whatever of them is pending when the lane is free runs as one batched
 * launch on the lane's own stream, beside the slots, and requests arriving
 * meanwhile form the next batch.  A fit's result is the same whichever batch
 * it joins (each fit is computed on its own); a batch-lane result differs
 * from the same fit run by cp_fit within the batched path's tolerance (its
 * tensor pass accumulates in FP64 without matrix cores).  The
 * caller keeps ownership of each request's tensor and factors until its
 * result has been polled.  Results do not depend on what else is running. */
typedef struct dgn_server dgn_server;

typedef struct dgn_request {
  dgn_tensor Y;
  int32_t R;
  double mu0;          /* > 0 as given, <= 0 tau rule */
  double tol;
  int32_t max_iters;
  void* A[DGN_MAX_ORDER]; /* device FP64 factors: in start, out result */
  uint64_t tag;        /* caller's tag, returned with the result */
} dgn_request;

typedef struct dgn_result {
  uint64_t id;
  uint64_t tag;
  int32_t status;      /* dgn_status of the fit */
  dgn_fit_info info;
  double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock */
  int32_t lane;        /* 0: ran in a slot (cp_fit); 1: ran in the batch lane (cp_fit_batched) */
  int32_t batch_size;  /* fits in the batched launch that ran it (1 for a slot) */
} dgn_result;

/* max_slots concurrent fits (1..64); opts as for cp_fit (may be NULL). */
dgn_status dgn_server_create(dgn_server** out, int32_t device, size_t budget_bytes,
                             int32_t max_slots, const dgn_opts* opts);
/* Queue a request; never blocks.  DGN_EBUSY if its workspace can never fit
 * the budget, DGN_EINVAL on a bad shape.  *id identifies the result. */
dgn_status dgn_server_submit(dgn_server* srv, const dgn_request* req, uint64_t* id);
/* Move up to max finished results into out; *n receives the count. */
dgn_status dgn_server_poll(dgn_server* srv, dgn_result* out, int32_t max, int32_t* n);
/* Block until nothing is queued or running. */
dgn_status dgn_server_wait_idle(dgn_server* srv);
/* Current arena bytes in use, running fits, queued requests (any may be NULL). */
dgn_status dgn_server_stats(dgn_server* srv, size_t* in_use, int32_t* running, int32_t* queued);
/* Seconds on the server clock (the clock of t_submit / t_admit / t_done). */
double dgn_server_now(const dgn_server* srv);
dgn_status dgn_server_destroy(dgn_server* srv);

/* Per-phase GPU time of the last cp_fit call made with opts->timing != 0,
 * from HIP events recorded on that call's stream around each phase of every
 * executed trial.  ms_out[k] (k < n <= DGN_NUM_PHASES) receives the total
 * milliseconds of phase k; *trials the number of trials summed.  Phases:
 * 0 Gamma / damped inverses / gradient rows / right-hand side,
 * 1 assembly of the NR^2 system (with the block-1 Schur update),
 * 2 Cholesky factorisation and triangular solves,
 * 3 factor update and candidate Gram matrices,
 * 4 tensor pass at the candidate (all-mode MTTKRP or residual pass),
 * 5 damping control and commit. */
#define DGN_NUM_PHASES 6
dgn_status dgn_last_phase_times(const dgn_ctx* ctx, double* ms_out, int32_t n, int32_t* trials);

#ifdef __cplusplus
}
#endif

#endif /* DGN_H */
