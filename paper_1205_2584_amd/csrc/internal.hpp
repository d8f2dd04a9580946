// Host-side launchers shared between the kernel files and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace dgn {

enum class YType { F64 = 0, F32 = 1, BF16 = 2, C64 = 3, C128 = 4 };

// Launch plan of the one-pass tensor kernel (all-mode MTTKRP, optionally on
// the residual E = Y - Y_hat formed on the fly).
struct PassPlan {
  int tiles_i, tiles_j;  // 64-row / 64-column tiles of the I_1 x I_2 slab
  int n_qc, q_per;       // chunks of the trailing index q and slabs per chunk
  long long Q;           // prod_{k>=2} I_k
  size_t m0_elems, m1_elems, t_elems, e2_elems;  // partial-sum buffers (compute type)
  size_t tbuf_elems;     // FP64 Q x R buffer (N >= 4 only)
  int tc_bytes;          // 8 (FP64 pass) or 4 (FP32 accumulation)
  int mfma;              // 1 when the MFMA kernel is used
};

PassPlan plan_pass(const Shape& s, YType yt);

struct PassBuffers {
  void* m0part;
  void* m1part;
  void* tpart;
  double* e2part;
  double* tbuf;
};

// M (stacked FP64, I_n x R per mode) = MTTKRP of Y (resid = false) or of
// E = Y - Y_hat (resid = true) at the stacked FP64 factors A.  With resid,
// e2out[0] receives sum(E^2).  Returns hipSuccess or the launch error.
// Work folded into the pass's final reduction launch (fits only):
// ipart receives ceil(I_1 R / 64) partial sums of <A_1, M_1> (the error of
// the candidate is ||Y||^2 - 2 <A_1, M_1> + ||Y_hat||^2); with rowpart, the
// row-chunk Gram partials of the update are summed into gout (N R^2) and its
// two per-row scalars into gscal (what launch_update_reduce does).
struct PassFold {
  double* ipart = nullptr;
  const double* rowpart = nullptr;
  int chunks = 0, stride = 0;
  double* gout = nullptr;
  double* gscal = nullptr;
};
hipError_t launch_tensor_pass(const Shape& s, YType yt, const void* Y, const double* A, bool resid,
                              const PassPlan& p, const PassBuffers& b, double* M, double* e2out,
                              const int* stop, hipStream_t st, const PassFold* fold = nullptr);

// sum(y^2) over n elements of Y in FP64.
hipError_t launch_norm2(YType yt, const void* Y, long long n, double* part, int nparts, double* out,
                        hipStream_t st);

// ---- small FP64 kernels (R x R objects, factor rows) ------------------------
struct SmallBuffers {
  double *C, *Cc;        // Gram matrices (current / candidate), N R^2
  double *Gam, *Gt, *X, *Lc;  // Gamma^(n), (Gamma^(n)+mu I)^-1, X X^T = Gt, L L^T = C; N R^2 each
  double *G, *P;         // gradient blocks and G~ g blocks, stacked T x R
  double *wpart;         // N x chunks x R^2
  double *w, *z, *y, *u, *f, *Q;  // N R^2 each (y, z padded)
  double *Tnm;           // N x N x R x R^2 (T_nm[i, a + d R])
  double *rowpart;       // N x chunks x (R^2 + 4) partial Grams and scalars
  double *scal;          // per-trial scalars: denom, ||da||^2, ||g||^2, ||M||^2
  double *ipart;         // pieces of <A_1, M_1> from the pass's reduction, ceil(I_max R / 64)
};

int row_chunks(const Shape& s);  // 64-row chunks per mode

hipError_t launch_gram(const Shape& s, const double* A, const SmallBuffers& b, double* Cout,
                       const int* stop, hipStream_t st);
hipError_t launch_gamma(const Shape& s, const double* C, double mu_host, const FitState* state,
                        const SmallBuffers& b, int* singular, const int* stop, hipStream_t st);
// G, P and the row-chunk partials of w (and, with with_tnm, the T_nm of the
// NR^2 assembly in the same launch).
hipError_t launch_pw(const Shape& s, const double* A, const double* M, bool resid,
                     const SmallBuffers& b, bool with_tnm, const int* stop, hipStream_t st);
// w, ||G||^2, ||M||^2 from the partials, and z = W^T K w.
hipError_t launch_wz(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st);
hipError_t launch_u(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st);
hipError_t launch_fq(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st);
// A_c = A + P - A Q_n; partial Grams of A_c and the gain-ratio denominator.
// Ac = A + da; da itself also into da_out when it is not NULL.
hipError_t launch_update(const Shape& s, const double* A, double* Ac, const SmallBuffers& b,
                         double mu_host, const FitState* state, const int* stop, hipStream_t st,
                         double* da_out = nullptr);
hipError_t launch_update_reduce(const Shape& s, const SmallBuffers& b, double* scal_out,
                                const int* stop, hipStream_t st);
// ALS update of mode n (eq. ALS): A_n = M_n Gt_n, with Gt_n = Gamma^(n)^-1 as
// left in b.Gt by launch_gamma at mu = 0.
hipError_t launch_als_rows(const Shape& s, int n, const double* M, const SmallBuffers& b, double* A,
                           hipStream_t st);

// ---- NR^2 system (trailing Schur complement, Cholesky, solves) --------------
struct SysPlan {
  int R2;       // R^2
  int nt;       // (N-1) R^2, trailing size
  int ntp;      // nt padded to a multiple of 64
  int Tt;       // ntp / 64 tiles
  int lds;      // leading dimension of the trailing matrix: ntp + 64 (RHS row tile)
};
SysPlan plan_sys(const Shape& s);

struct SysBuffers {
  double* St;   // lds x ntp, column-major; rows ntp.. hold the right-hand side row
  double* B;    // ntp x R^2, the first block column of S below the identity block
  double* yt;   // ntp
  double* Ld;   // Tt tiles of 64 x 64 (column-major, leading dimension 64): the factored
                // diagonal tiles L(k, k). They live apart from St so that, while phase k
                // runs, every workgroup still reads the unfactored tile (k, k) from St.
  double* Li;   // Tt tiles of 64 x 64 (row-major): L(k, k)^-1, for the backward
                // substitution of systems too large for the Gauss-Jordan elimination
};

hipError_t launch_sys_assemble(const Shape& s, const SysPlan& p, const SmallBuffers& b,
                               const SysBuffers& y, const int* stop, hipStream_t st);
// structured_b: y_1 = z_1 - B^T y_t from the structure of B (real systems, R <= 32,
// assembled without B); otherwise from B itself.
hipError_t launch_sys_factor_solve(const Shape& s, const SysPlan& p, const SmallBuffers& b,
                                   const SysBuffers& y, int* singular, const int* stop,
                                   hipStream_t st, bool structured_b = false);
// The tiled Cholesky of the lower tiles of y.St with the right-hand-side row
// (forward substitution inside) and the backward substitution, carried along
// the phases as Gauss-Jordan elimination (upper tiles of y.St), into y.yt; any
// system size with the SysPlan layout.
hipError_t launch_sys_factor_solve_core(const SysPlan& p, const SysBuffers& y, int* singular, const int* stop,
                                        hipStream_t st);

// ---- explicit-Hessian dGN step (Section 3; the comparison baseline) -----------
// System of the RT parameters: nt = R T, padded to 64.
SysPlan plan_sys_explicit(const Shape& s);
// H + mu I (lower tiles) and the gradient G (stacked T x R, as the right-hand-side row) into St.
hipError_t launch_explicit_system(const Shape& s, const SysPlan& p, const double* A, const double* C,
                                  const double* G, double mu, double* St, hipStream_t st);
// Ac = A + da; scal[0] = da^T (G + mu da), scal[1] = ||da||^2.
hipError_t launch_explicit_update(const SysPlan& p, const double* A, const double* da, const double* G,
                                  double mu, double* Ac, double* scal, hipStream_t st);

// The assemble phase in two parts so that the complex path can write its own
// (embedded) sub-blocks in between: identity / zero fill, then RHS row and SYRK.
hipError_t launch_sys_fill(const SysPlan& p, const SysBuffers& y, const int* stop, hipStream_t st);
hipError_t launch_sys_rhs_syrk(const SysPlan& p, const double* z, const SysBuffers& y, const int* stop,
                               hipStream_t st);

// ---- complex path (Section 5): FP64 complex factors, interleaved (re, im) ------
constexpr int kMaxRankC = 32;
PassPlan plan_pass_c(const Shape& s);
// The real embedding of the complex trailing system: R2 = 2 R^2, nt = 2 (N-1) R^2.
SysPlan plan_sys_c(const Shape& s);
hipError_t launch_tensor_pass_c(const Shape& s, bool y64, const void* Y, const double* A, bool resid,
                                const PassPlan& p, const PassBuffers& b, double* M, double* e2out,
                                const int* stop, hipStream_t st);
hipError_t launch_inner_c(const Shape& s, const double* A, const double* M, double* out, hipStream_t st);
hipError_t launch_gram_c(const Shape& s, const double* A, const SmallBuffers& b, double* Cout,
                         const int* stop, hipStream_t st);
hipError_t launch_small_pre_c(const Shape& s, const double* A, const double* M, bool resid, double mu_host,
                              const FitState* state, const SmallBuffers& b, int* singular,
                              const int* stop, hipStream_t st);
hipError_t launch_subblock_c(const Shape& s, const SysPlan& p, const SmallBuffers& b, const SysBuffers& y,
                             const int* stop, hipStream_t st);
hipError_t launch_small_post_c(const Shape& s, const double* A, double* Ac, const SmallBuffers& b,
                               double mu_host, const FitState* state, const int* stop, hipStream_t st, double* da_out = nullptr);
// Gamma_n, the Cholesky of Gamma_n + mu I and Gt_n = (Gamma_n + mu I)^-1 for every mode (complex).
hipError_t launch_gamma_c(const Shape& s, const double* C, double mu_host, const FitState* state,
                          const SmallBuffers& b, int* singular, const int* stop, hipStream_t st);
// Complex ALS update of mode n: A_n = M_n conj(Gt_n), Gt_n = Gamma^(n)^-1 from launch_gamma_c at mu = 0.
hipError_t launch_als_rows_c(const Shape& s, int n, const double* M, const SmallBuffers& b, double* A,
                             hipStream_t st);

// ---- fit control -------------------------------------------------------------
// cs: doubles per element of the factor, MTTKRP and Gram arrays (1 real, 2 complex).
hipError_t launch_fit_init(const Shape& s, const double* A, const double* M, const double* C,
                           bool resid, const double* e2, double mu0, double tau, FitState* state,
                           hipStream_t st, int cs = 1);
hipError_t launch_refresh(const Shape& s, const double* e2, FitState* state, hipStream_t st);
hipError_t launch_err2(const Shape& s, const double* A, const double* M, const double* C, bool resid,
                       const double* e2, const double* ynorm2_pass, double* out, hipStream_t st);
// ipart (nip values): <A_1, M_1> in pieces from the pass (PassFold); null:
// the inner product is formed here from Ac and Mc.
hipError_t launch_control(const Shape& s, const double* Ac, const double* Mc, const double* Cc,
                          bool resid, const double* e2, const double* scal, FitState* state,
                          int trial, hipStream_t st, int cs = 1, const double* ipart = nullptr,
                          int nip = 0);
hipError_t launch_commit(const Shape& s, double* A, const double* Ac, double* M, const double* Mc,
                         double* C, const double* Cc, const FitState* state, int trial,
                         hipStream_t st, int cs = 1);

// ---- batched small fits (one block per fit per trial) ---------------------------
struct BFit {
  const void* Y;
  int dtype;  // 0 = FP64, 1 = FP32
  int I[3];
  int R;
  double mu0;
  double *A, *Ac, *M, *Mc, *G, *P, *C, *Cc;  // per-fit workspace
  double* Ain[3];                             // caller's factors
  FitState* st;
};

struct BatchCfg {
  double tol, tau, resid_switch;
  int max_iters, normalize, mu_rule;
  int* nstopped;
};

bool batched_supported(int order, const int64_t* dims, int R);
size_t batched_fit_doubles(const int* I, int R);
hipError_t launch_batched_init(BFit* fits, int nfits, const BatchCfg& cfg, hipStream_t st);
hipError_t launch_batched_trial(BFit* fits, int nfits, const BatchCfg& cfg, hipStream_t st);
hipError_t launch_batched_final(BFit* fits, int nfits, hipStream_t st);
// Persistent form: `blocks` blocks drain a queue of the fits (queue: one int of
// device memory, reset on the stream first), each running a fit from its
// initial state through at most `ntrials` trials; copy_out writes the result
// factors to the caller's buffers.
hipError_t launch_batched_persistent(BFit* fits, int nfits, const int* order, int* queue, const BatchCfg& cfg,
                                     int blocks, int ntrials, bool copy_out, hipStream_t st);

// ---- iterative NR^2 solve (conjugate gradients on the structured SPD form) ----
bool cg_supported(const Shape& s);  // N <= 4, R <= 32
// y = S^-1 z by CG from b.C, b.X, b.Lc, b.z into b.y; cgf[0] = 1 when the
// direct solve can be skipped (see the kernel for the other counters); mu from
// state when state != NULL, which also carries the retry rule of a fit.
hipError_t launch_cg(const Shape& s, const SmallBuffers& b, double tol, int maxit, FitState* state, double mu_host,
                     int* cgf, const int* stop, hipStream_t st);
// The same for the complex step (Hermitian S, embedded z and y), N <= 4, R <= 16.
bool cg_supported_c(const Shape& s);
hipError_t launch_cg_c(const Shape& s, const SmallBuffers& b, double tol, int maxit, FitState* state, double mu_host,
                       int* cgf, const int* stop, hipStream_t st);

// ---- mode-n singular vectors (SVD initialisation) ---------------------------
// Y viewed for mode n as (P, I, Q): element (p, i, q) at p + P (i + I q).
struct GramPlan {
  long long P, Q;
  int I, ntile;            // mode size, lower 128 x 128 tiles of G_n
  long long nchunk, cps;   // summation chunks of 32, chunks per split
  int S;                   // splits of the summation (partial tiles per tile)
};
GramPlan plan_gram(const Shape& s, int n);
size_t gram_part_doubles(const Shape& s);  // partial-tile buffer for any mode

// Per-mode buffers of the subspace iteration: G_n (Ip x Ip), Q_n and Z_n
// (Ip x bp, column-major, leading dimension Ip; Ip = I_n rounded up to 64,
// bp = b rounded up to 16) and the output factor A_n (I_n x R).
struct SvdModes {
  int N, b, bp, R;
  int I[kMaxOrder], Ip[kMaxOrder];
  double* G[kMaxOrder];
  double* Q[kMaxOrder];
  double* Z[kMaxOrder];
  double* A[kMaxOrder];
  int blk0[kMaxOrder + 1];  // first block of each mode in the Z = G Q launch
};

// G (leading dimension ld) = Y_(n) Y_(n)^T on rows/columns < lim (rows and
// columns in [I_n, lim) get zeros); part holds gram_part_doubles(s) doubles.
hipError_t launch_mode_gram(const Shape& s, int n, const void* Y, YType yt, double* part, double* G, long long ld,
                            int lim, hipStream_t st);
// Complex tensors: the Hermitian Gram from the real Gram of the interleaved
// rows (Gp: (2 I_n)^2 doubles), into its real embedding E (2 I_n x 2 I_n,
// leading dimension lde) and/or the interleaved complex Gc (I_n x I_n).
GramPlan plan_gram_c(const Shape& s, int n);
size_t gram_part_doubles_c(const Shape& s);
hipError_t launch_mode_gram_c(const Shape& s, int n, const void* Y, YType yt, double* part, double* Gp,
                              double* E, long long lde, double* Gc, hipStream_t st);
struct CxFactors {
  double* A[kMaxOrder];  // interleaved complex I_n x R outputs
};
// Complex SVD initialisation on the real embeddings: m describes the doubled
// problem (I = 2 I_n, b = 2 block, R = 2 R, A = real scratch 2 I_n x 2 R),
// svr N x 2R scratch; the complex factors go to out, sv (N x R) when not NULL.
hipError_t launch_svd_init_c(const Shape& s, const void* Y, YType yt, SvdModes m, CxFactors out, double* Gp,
                             const double* omega, int iters, double* part, double* sigma, double* svr, double* sv,
                             int* bad, hipStream_t st);
// The whole SVD initialisation; sigma: N doubles, sv: N x R or NULL, *bad
// raised on a Cholesky breakdown of the orthonormalisation.
hipError_t launch_svd_init(const Shape& s, const void* Y, YType yt, SvdModes m, const double* omega, int iters,
                           double* part, double* sigma, double* sv, int* bad, hipStream_t st);

}  // namespace dgn
