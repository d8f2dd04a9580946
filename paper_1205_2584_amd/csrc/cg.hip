// Iterative solve of the NR^2 system of the fast step: conjugate gradients on
// the SPD form S y = z, S = I + W^T K W (W = blkdiag(X_n (x) L_n),
// X_n X_n^T = (Gamma_n + mu I)^-1, L_n L_n^T = C_n), with S never formed.
// The product uses the Kronecker structure of W and the permuted-diagonal
// blocks K_nm = P_R diag(vec Gamma_nm) of K (Section 4.3):
//   U_m = L_m Y_m X_m^T,   V_n = sum_{m != n} Gamma_nm .* U_m,
//   (S y)_n = Y_n + L_n^T V_n^T X_n,          Y_n = unvec(y_n) (R x R),
// which costs O(N R^3 + N^2 R^2) flops against O(N^2 R^4) for the formed
// matrix.  Section 4.3 suggests an iterative solver on the structured system;
// S is symmetric positive definite, so CG applies.
//
// One workgroup of 1024 threads holds every operand in LDS (N <= 4, R <= 32,
// padded to 32 with zeros); the four R x R products per mode run on FP64 MFMA.
// Thread t owns entry (t % 32, t / 32) of every mode's R x R block of the CG
// vectors, so the Hadamard step and the vector updates need no exchange.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int CN = 4;       // modes held
constexpr int CR = 32;      // padded rank
constexpr int CS = CR + 1;  // LDS row stride

// out(m, r, c) = sum_k fa(m, r, k) fb(m, k, c) over k < 32 for the 32 x 32
// products of modes m < N; wave w takes the 16 x 16 output blocks w, w + 16, ...
// (v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16], B[l / 16][l % 16],
// result rows l / 16 + 4v, column l % 16).
template <class FA, class FB, class FO>
__device__ __forceinline__ void gemm32(int N, FA fa, FB fb, FO fo) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int bidx = w; bidx < 4 * N; bidx += 16) {
    const int m = bidx >> 2, r0 = 16 * ((bidx >> 1) & 1), c0 = 16 * (bidx & 1);
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < CR; k += 4) {
      const int kk = k + (lane >> 4);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa(m, r0 + (lane & 15), kk), fb(m, kk, c0 + (lane & 15)), acc, 0,
                                                 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) fo(m, r0 + (lane >> 4) + 4 * v, c0 + (lane & 15), acc[v]);
  }
}

// Early exit of a solve that will not converge within the cap: every 10
// iterations from the 20th, the mean reduction of ||r||^2 per iteration so far
// is extrapolated; when the goal lies beyond twice maxit the solve gives up (the
// direct solve then runs), so a hopeless attempt costs about 20 iterations
// rather than maxit.  Uniform across the workgroup (scalars from block sums).
__device__ __forceinline__ bool give_up(int it, double rn, double rr0, double goal, int maxit) {
  if (it < 20 || it % 10 != 0 || !(rn > 0.0) || !(rn < rr0)) return it >= 20 && it % 10 == 0 && !(rn < rr0);
  const double per = log(rn / rr0) / it;  // < 0
  const double need = log(goal / rn) / per;
  return it + need > 2.0 * maxit;  // twice the cap: CG often speeds up once the outliers are resolved
}

// Sum over the workgroup with a single barrier: the callers alternate two
// scratch arrays, and every reuse of one is separated from its previous reads
// by the barriers of the product phases.
__device__ __forceinline__ double block_sum1(double v, double* scratch) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  sync_block();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += scratch[i];
  return s;
}

// cgf: [0] 1 when the direct solve is to be skipped (converged, or the fit has
// stopped), [2] this solve's iterations, [3] solves that converged, [4] their
// iterations summed.  A solve that cannot reach the goal within maxit at its
// rate so far gives up early (give_up).  Inside a fit (state != NULL) the first failed solve
// records its damping in the state and CG is not tried again in that fit, so a
// fit loses at most one capped attempt.
__global__ __launch_bounds__(1024) void k_cg(Shape s, const double* __restrict__ C, const double* __restrict__ X,
                                             const double* __restrict__ Lc, const double* __restrict__ z,
                                             double* __restrict__ y, double tol, int maxit, FitState* state,
                                             double mu_host, int* cgf, const int* stop) {
  __shared__ double Ls[CN][CR][CS];
  __shared__ double Xs[CN][CR][CS];
  __shared__ double Ps[CN][CR][CS];
  __shared__ double Ts[CN][CR][CS];
  __shared__ double red[16];
  __shared__ double red_a[16];
  __shared__ double red_b[16];
  if (stopped(stop)) {
    if (threadIdx.x == 0) cgf[0] = 1;
    return;
  }
  const double mu = state ? state->mu : mu_host;
  if (state && state->cg_mu_fail > 0.0) {
    if (threadIdx.x == 0) cgf[0] = 0;
    return;
  }
  const int N = s.N, R = s.R, R2 = R * R, t = threadIdx.x;
  for (int e = t; e < CN * CR * CR; e += 1024) {
    const int n = e / (CR * CR), rem = e % (CR * CR), i = rem % CR, j = rem / CR;
    const bool in = n < N && i < R && j < R;
    Ls[n][i][j] = in ? Lc[(long long)n * R2 + i + j * R] : 0.0;
    Xs[n][i][j] = in ? X[(long long)n * R2 + i + j * R] : 0.0;
  }
  const int gi = t % CR, gj = t / CR;
  const bool gin = gi < R && gj < R;
  // Gamma_nm at (gi, gj): the Hadamard product of C_k over k not in {n, m}
  double cv[CN];
#pragma unroll
  for (int k = 0; k < CN; ++k) cv[k] = (k < N && gin) ? C[(long long)k * R2 + gi + gj * R] : 0.0;
  double g[CN][CN];
#pragma unroll
  for (int n = 0; n < CN; ++n)
#pragma unroll
    for (int m = 0; m < CN; ++m) {
      // zero for the modes n, m >= N that only pad the arrays, so that their
      // entries of the CG vectors stay zero
      double p = (gin && n < N && m < N) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < CN; ++k)
        if (k < N && k != n && k != m) p *= cv[k];
      g[n][m] = p;
    }
  double xv[CN], rv[CN], pv[CN];
  double zz = 0.0;
#pragma unroll
  for (int n = 0; n < CN; ++n) {
    const double zv = (n < N && gin) ? z[(long long)n * R2 + gi + gj * R] : 0.0;
    xv[n] = 0.0;
    rv[n] = zv;
    pv[n] = zv;
    zz += zv * zv;
  }
  double rr = block_sum(zz, red);
  const double rr0 = rr;
  const double goal = tol * tol * rr;  // stop at ||r|| <= tol ||z||
  bool conv = rr <= goal;
  int it = 0;
  while (!conv && it < maxit && isfinite(rr)) {
#pragma unroll
    for (int n = 0; n < CN; ++n) Ps[n][gi][gj] = pv[n];
    sync_block();
    // T_m = L_m P_m
    gemm32(
        N, [&](int m, int r, int k) { return Ls[m][r][k]; }, [&](int m, int k, int c) { return Ps[m][k][c]; },
        [&](int m, int r, int c, double v) { Ts[m][r][c] = v; });
    sync_block();
    // U_m = T_m X_m^T (into Ps)
    gemm32(
        N, [&](int m, int r, int k) { return Ts[m][r][k]; }, [&](int m, int k, int c) { return Xs[m][c][k]; },
        [&](int m, int r, int c, double v) { Ps[m][r][c] = v; });
    sync_block();
    // V_n = sum_{m != n} Gamma_nm .* U_m (into Ts), entry (gi, gj) of every mode
    {
      double u[CN];
#pragma unroll
      for (int m = 0; m < CN; ++m) u[m] = Ps[m][gi][gj];
#pragma unroll
      for (int n = 0; n < CN; ++n) {
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < CN; ++m)
          if (m != n) v += g[n][m] * u[m];
        Ts[n][gi][gj] = v;
      }
    }
    sync_block();
    // W_n = V_n^T X_n (into Ps)
    gemm32(
        N, [&](int m, int r, int k) { return Ts[m][k][r]; }, [&](int m, int k, int c) { return Xs[m][k][c]; },
        [&](int m, int r, int c, double v) { Ps[m][r][c] = v; });
    sync_block();
    // O_n = L_n^T W_n (into Ts); (S p)_n = P_n + O_n
    gemm32(
        N, [&](int m, int r, int k) { return Ls[m][k][r]; }, [&](int m, int k, int c) { return Ps[m][k][c]; },
        [&](int m, int r, int c, double v) { Ts[m][r][c] = v; });
    sync_block();
    double ap[CN];
    double pap = 0.0;
#pragma unroll
    for (int n = 0; n < CN; ++n) {
      ap[n] = n < N ? pv[n] + Ts[n][gi][gj] : 0.0;
      pap += pv[n] * ap[n];
    }
    pap = block_sum1(pap, red_a);
    if (!(pap > 0.0)) break;  // not positive definite in finite precision: leave it to the direct solve
    const double alpha = rr / pap;
    double rn = 0.0;
#pragma unroll
    for (int n = 0; n < CN; ++n) {
      xv[n] += alpha * pv[n];
      rv[n] -= alpha * ap[n];
      rn += rv[n] * rv[n];
    }
    rn = block_sum1(rn, red_b);
    ++it;
    conv = rn <= goal;
    if (!conv && give_up(it, rn, rr0, goal, maxit)) break;
    const double beta = rn / rr;
    rr = rn;
#pragma unroll
    for (int n = 0; n < CN; ++n) pv[n] = rv[n] + beta * pv[n];
  }
  if (conv) {
#pragma unroll
    for (int n = 0; n < CN; ++n)
      if (n < N && gin) y[(long long)n * R2 + gi + gj * R] = xv[n];
  }
  if (t == 0) {
    cgf[0] = conv ? 1 : 0;
    cgf[2] = it;
    if (conv) {
      cgf[3] += 1;
      cgf[4] += it;
    } else if (state) {
      state->cg_mu_fail = mu;
    }
  }
}

// Complex tensors (Section 5): the Hermitian positive definite S = I + W^H K W
// of the complex step, S_nm[a + bR, c + dR] = sum_{j,i} conj(X_n[j,b]) L_m[j,c]
// Gamma_nm[j,i] conj(L_n[i,a]) X_m[i,d], applied as
//   U_m = L_m Y_m X_m^T,  V_n = sum_{m != n} Gamma_nm .* U_m,
//   (S y)_n = Y_n + L_n^H V_n^T conj(X_n).
// Here R <= 16: thread t owns entry (t % 16, (t / 16) % 16) of mode t / 256, and
// wave m < N computes mode m's 16 x 16 complex products (four real MFMA chains).
// z and y use the embedded layout of the direct solve: [Re z_1, Im z_1, Re z_t, Im z_t].
constexpr int QR = 16;
constexpr int QS = QR + 1;

template <class FA, class FB, class FO>
__device__ __forceinline__ void cgemm16(int N, FA fa, FB fb, FO fo) {
  const int lane = threadIdx.x & 63, m = threadIdx.x >> 6;
  if (m >= N) return;
  v4d ar = v4d{0.0, 0.0, 0.0, 0.0}, ai = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < QR; k += 4) {
    const int kk = k + (lane >> 4);
    double a_re, a_im, b_re, b_im;
    fa(m, lane & 15, kk, a_re, a_im);
    fb(m, kk, lane & 15, b_re, b_im);
    ar = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re, b_re, ar, 0, 0, 0);
    ar = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_im, b_im, ar, 0, 0, 0);
    ai = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re, b_im, ai, 0, 0, 0);
    ai = __builtin_amdgcn_mfma_f64_16x16x4f64(a_im, b_re, ai, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) fo(m, (lane >> 4) + 4 * v, lane & 15, ar[v], ai[v]);
}

__device__ __forceinline__ long long emb_re(int n, int e, int R2, int N) {
  return n == 0 ? e : 2LL * R2 + (long long)(n - 1) * R2 + e;
}
__device__ __forceinline__ long long emb_im(int n, int e, int R2, int N) {
  return n == 0 ? (long long)R2 + e : 2LL * R2 + (long long)(N - 1) * R2 + (long long)(n - 1) * R2 + e;
}

__global__ __launch_bounds__(1024) void k_cg_c(Shape s, const double* __restrict__ C, const double* __restrict__ X,
                                               const double* __restrict__ Lc, const double* __restrict__ z,
                                               double* __restrict__ y, double tol, int maxit, FitState* state,
                                               double mu_host, int* cgf, const int* stop) {
  __shared__ double Lr[CN][QR][QS], Li[CN][QR][QS], Xr[CN][QR][QS], Xi[CN][QR][QS];
  __shared__ double Pr[CN][QR][QS], Pi[CN][QR][QS], Tr[CN][QR][QS], Ti[CN][QR][QS];
  __shared__ double red[16], red_a[16], red_b[16];
  if (stopped(stop)) {
    if (threadIdx.x == 0) cgf[0] = 1;
    return;
  }
  const double mu = state ? state->mu : mu_host;
  if (state && state->cg_mu_fail > 0.0) {
    if (threadIdx.x == 0) cgf[0] = 0;
    return;
  }
  const int N = s.N, R = s.R, R2 = R * R, t = threadIdx.x;
  const int gn = t >> 8, gi = t & 15, gj = (t >> 4) & 15;
  const bool act = gn < N && gi < R && gj < R;
  const int e = gi + gj * R;
  Lr[gn][gi][gj] = act ? Lc[2 * ((long long)gn * R2 + e)] : 0.0;
  Li[gn][gi][gj] = act ? Lc[2 * ((long long)gn * R2 + e) + 1] : 0.0;
  Xr[gn][gi][gj] = act ? X[2 * ((long long)gn * R2 + e)] : 0.0;
  Xi[gn][gi][gj] = act ? X[2 * ((long long)gn * R2 + e) + 1] : 0.0;
  // Gamma_{gn,m} at (gi, gj): complex product of C_k over k not in {gn, m}
  double cre[CN], cim[CN];
#pragma unroll
  for (int k = 0; k < CN; ++k) {
    const bool in = k < N && gi < R && gj < R;
    cre[k] = in ? C[2 * ((long long)k * R2 + e)] : 0.0;
    cim[k] = in ? C[2 * ((long long)k * R2 + e) + 1] : 0.0;
  }
  double gre[CN], gim[CN];
#pragma unroll
  for (int m = 0; m < CN; ++m) {
    double pr = (act && m < N && m != gn) ? 1.0 : 0.0, pi = 0.0;
#pragma unroll
    for (int k = 0; k < CN; ++k)
      if (k < N && k != gn && k != m) {
        const double nr = pr * cre[k] - pi * cim[k];
        pi = pr * cim[k] + pi * cre[k];
        pr = nr;
      }
    gre[m] = pr;
    gim[m] = pi;
  }
  double xr = 0.0, xi = 0.0;
  double rr_ = act ? z[emb_re(gn, e, R2, N)] : 0.0, ri = act ? z[emb_im(gn, e, R2, N)] : 0.0;
  double pr = rr_, pi = ri;
  double rr = block_sum(rr_ * rr_ + ri * ri, red);
  const double rr0 = rr;
  const double goal = tol * tol * rr;
  bool conv = rr <= goal;
  int it = 0;
  while (!conv && it < maxit && isfinite(rr)) {
    Pr[gn][gi][gj] = pr;
    Pi[gn][gi][gj] = pi;
    sync_block();
    // T_m = L_m P_m
    cgemm16(
        N, [&](int m, int r, int k, double& a, double& b) { a = Lr[m][r][k]; b = Li[m][r][k]; },
        [&](int m, int k, int c, double& a, double& b) { a = Pr[m][k][c]; b = Pi[m][k][c]; },
        [&](int m, int r, int c, double a, double b) { Tr[m][r][c] = a; Ti[m][r][c] = b; });
    sync_block();
    // U_m = T_m X_m^T (into P)
    cgemm16(
        N, [&](int m, int r, int k, double& a, double& b) { a = Tr[m][r][k]; b = Ti[m][r][k]; },
        [&](int m, int k, int c, double& a, double& b) { a = Xr[m][c][k]; b = Xi[m][c][k]; },
        [&](int m, int r, int c, double a, double b) { Pr[m][r][c] = a; Pi[m][r][c] = b; });
    sync_block();
    // V_n = sum_{m != n} Gamma_nm .* U_m (into T)
    {
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int m = 0; m < CN; ++m) {
        const double ur = Pr[m][gi][gj], ui = Pi[m][gi][gj];
        vr += gre[m] * ur - gim[m] * ui;
        vi += gre[m] * ui + gim[m] * ur;
      }
      Tr[gn][gi][gj] = vr;
      Ti[gn][gi][gj] = vi;
    }
    sync_block();
    // W_n = V_n^T conj(X_n) (into P)
    cgemm16(
        N, [&](int m, int r, int k, double& a, double& b) { a = Tr[m][k][r]; b = Ti[m][k][r]; },
        [&](int m, int k, int c, double& a, double& b) { a = Xr[m][k][c]; b = -Xi[m][k][c]; },
        [&](int m, int r, int c, double a, double b) { Pr[m][r][c] = a; Pi[m][r][c] = b; });
    sync_block();
    // O_n = L_n^H W_n (into T); (S p)_n = P_n + O_n
    cgemm16(
        N, [&](int m, int r, int k, double& a, double& b) { a = Lr[m][k][r]; b = -Li[m][k][r]; },
        [&](int m, int k, int c, double& a, double& b) { a = Pr[m][k][c]; b = Pi[m][k][c]; },
        [&](int m, int r, int c, double a, double b) { Tr[m][r][c] = a; Ti[m][r][c] = b; });
    sync_block();
    const double apr = act ? pr + Tr[gn][gi][gj] : 0.0, api = act ? pi + Ti[gn][gi][gj] : 0.0;
    const double pap = block_sum1(pr * apr + pi * api, red_a);  // Re(p^H S p)
    if (!(pap > 0.0)) break;
    const double alpha = rr / pap;
    xr += alpha * pr;
    xi += alpha * pi;
    rr_ -= alpha * apr;
    ri -= alpha * api;
    const double rn = block_sum1(rr_ * rr_ + ri * ri, red_b);
    ++it;
    conv = rn <= goal;
    if (!conv && give_up(it, rn, rr0, goal, maxit)) break;
    const double beta = rn / rr;
    rr = rn;
    pr = rr_ + beta * pr;
    pi = ri + beta * pi;
  }
  if (conv && act) {
    y[emb_re(gn, e, R2, N)] = xr;
    y[emb_im(gn, e, R2, N)] = xi;
  }
  if (t == 0) {
    cgf[0] = conv ? 1 : 0;
    cgf[2] = it;
    if (conv) {
      cgf[3] += 1;
      cgf[4] += it;
    } else if (state) {
      state->cg_mu_fail = mu;
    }
  }
}

}  // namespace

bool cg_supported(const Shape& s) { return s.N <= CN && s.R <= CR; }

hipError_t launch_cg(const Shape& s, const SmallBuffers& b, double tol, int maxit, FitState* state, double mu_host,
                     int* cgf, const int* stop, hipStream_t st) {
  if (!cg_supported(s)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg, dim3(1), dim3(1024), 0, st, s, b.C, b.X, b.Lc, b.z, b.y, tol, maxit, state, mu_host, cgf,
                     stop);
  return hipGetLastError();
}

}  // namespace dgn

namespace dgn {

bool cg_supported_c(const Shape& s) { return s.N <= CN && s.R <= QR; }

hipError_t launch_cg_c(const Shape& s, const SmallBuffers& b, double tol, int maxit, FitState* state, double mu_host,
                       int* cgf, const int* stop, hipStream_t st) {
  if (!cg_supported_c(s)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_c, dim3(1), dim3(1024), 0, st, s, b.C, b.X, b.Lc, b.z, b.y, tol, maxit, state, mu_host,
                     cgf, stop);
  return hipGetLastError();
}

}  // namespace dgn
