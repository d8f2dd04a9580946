// Many small independent fits in one launch per trial.
//
// One 256-thread block owns one 3-way fit (R <= 8, every I_n <= 64) and runs
// a whole trial of Algorithm 1 for it: Gamma / damped inverses, the
// Jacobian-free products of Lemma 4.4, the NR^2 system in its SPD form
// S = I + W^T K W (block 1 eliminated first, the trailing (N-1)R^2 system
// factored in LDS with the right-hand side folded in as an extra row), the
// factor update, the tensor pass at the candidate (all-mode MTTKRP, FP32 for
// FP32 tensors, FP64 for FP64 ones; residual form after the switch), and the
// damping control of Section 4.5.  The same formulas as the large-problem
// kernels (small.hip, chol.hip, tensor_pass.hip, fit.hip); the trial kernel
// takes no per-launch arguments, so a run of trials is captured once in a
// hipGraph and replayed.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int BR = 8;          // max rank
constexpr int BR2 = BR * BR;   // 64
constexpr int BI = 64;         // max mode size
constexpr int BNT = 2 * BR2;   // max trailing system size (128)
constexpr int kPacked = (BNT + 1) * (BNT + 2) / 2;  // packed lower rows 0..BNT

__device__ __forceinline__ int pidx(int i, int j) { return i * (i + 1) / 2 + j; }

// Shared-memory layout (doubles).
struct Smem {
  double Cs[3][BR2], Gm[3][BR2], Gt[3][BR2], Xs[3][BR2], Ls[3][BR2], Qs[3][BR2];
  double w[3 * BR2], z[3 * BR2], y[3 * BR2], v[3 * BR2];
  double red[16];
  double scal[8];
  int flags[8];
  union {
    struct {
      double Sp[kPacked];
      double Bm[BNT][BR2];
      double Tb[BR * BR * BR];
    } sys;
    struct {
      double Ys[BI][BI + 1];  // Ys[j][i]
      double A0s[BI][BR + 1], A1s[BI][BR + 1];
      double cq[BR];
    } pass;
    struct {
      double V[3][BR2], T1[3][BR2];
    } rr;
  } u;
};

__device__ __forceinline__ int mode_of_row(const BFit& f, int row, int* i) {
  if (row < f.I[0]) { *i = row; return 0; }
  if (row < f.I[0] + f.I[1]) { *i = row - f.I[0]; return 1; }
  *i = row - f.I[0] - f.I[1];
  return 2;
}

__device__ __forceinline__ long long aoff(const BFit& f, int n) {
  long long o = 0;
  for (int k = 0; k < n; ++k) o += (long long)f.I[k] * f.R;
  return o;
}

// ---- tensor pass (one block, all modes) --------------------------------------
// Mout = MTTKRP of Y (or of E = Y - Y_hat when resid) at factors Ain; returns
// sum(E^2) (resid) or <Y, Y_hat> = sum(A_1 * M_1) (plain) to every thread.
template <typename TY>
__device__ double bpass(const BFit& f, const double* Ain, double* Mout, int resid, Smem& S) {
  const int t = threadIdx.x, lane = t & 63, rg = t >> 6;
  const int I0 = f.I[0], I1 = f.I[1], I2 = f.I[2], R = f.R;
  const TY* Y = static_cast<const TY*>(f.Y);
  const double* A0 = Ain;
  const double* A1 = Ain + (long long)I0 * R;
  const double* A2 = A1 + (long long)I1 * R;
  double* M0 = Mout;
  double* M1 = Mout + (long long)I0 * R;
  double* M2 = M1 + (long long)I1 * R;
  auto& P = S.u.pass;
  sync_block();
  for (int e = t; e < BI * BR; e += 256) {
    const int ii = e & 63, r = e >> 6;
    P.A0s[ii][r] = (ii < I0 && r < R) ? A0[ii + (long long)r * I0] : 0.0;
    P.A1s[ii][r] = (ii < I1 && r < R) ? A1[ii + (long long)r * I1] : 0.0;
  }
  double m0[2] = {0.0, 0.0}, m1[2] = {0.0, 0.0};
  double e2 = 0.0;
  // slice q of Y (and row q of A^(3)) is loaded into registers while slice
  // q - 1 is processed, every load of a slice issued before the first is used
  TY yv[16];
  double cv = 0.0;
  auto load_slice = [&](int q) {
    const long long base = (long long)I0 * I1 * q;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = t + 256 * k, ii = e & 63, jj = e >> 6;
      yv[k] = (ii < I0 && jj < I1) ? Y[base + ii + (long long)I0 * jj] : TY(0);
    }
    cv = (t < R) ? A2[q + (long long)t * I2] : 0.0;
  };
  if (I2 > 0) load_slice(0);
  for (int q = 0; q < I2; ++q) {
    sync_block();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = t + 256 * k, ii = e & 63, jj = e >> 6;
      P.Ys[jj][ii] = to_f64(yv[k]);
    }
    if (t < BR) P.cq[t] = cv;
    sync_block();
    if (q + 1 < I2) load_slice(q + 1);
    if (resid) {
      for (int e = t; e < BI * BI; e += 256) {
        const int ii = e & 63, jj = e >> 6;
        if (ii < I0 && jj < I1) {
          double yh = 0.0;
#pragma unroll
          for (int r = 0; r < BR; ++r)
            if (r < R) yh += P.A0s[ii][r] * (P.A1s[jj][r] * P.cq[r]);
          const double ev = P.Ys[jj][ii] - yh;
          e2 += ev * ev;
          P.Ys[jj][ii] = ev;
        }
      }
      sync_block();
    }
    double zp[2] = {0.0, 0.0}, wp[2] = {0.0, 0.0};
    // unrolled so that the LDS reads of several rows are in flight together
#pragma unroll 8
    for (int jj = 0; jj < I1; ++jj) {
      const double yv = P.Ys[jj][lane];
      zp[0] += yv * P.A1s[jj][rg];
      zp[1] += yv * P.A1s[jj][rg + 4];
    }
#pragma unroll 8
    for (int ii = 0; ii < I0; ++ii) {
      const double yv = P.Ys[lane][ii];
      wp[0] += yv * P.A0s[ii][rg];
      wp[1] += yv * P.A0s[ii][rg + 4];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int r = rg + 4 * k;
      const double c = P.cq[r];
      m0[k] += c * zp[k];
      m1[k] += c * wp[k];
      const double tv = wave_sum(P.A0s[lane][r] * zp[k]);
      if (lane == 0 && r < R) M2[q + (long long)r * I2] = tv;
    }
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = rg + 4 * k;
    if (r < R) {
      if (lane < I0) M0[lane + (long long)r * I0] = m0[k];
      if (lane < I1) M1[lane + (long long)r * I1] = m1[k];
    }
  }
  sync_block();
  double out;
  if (resid) {
    out = block_sum(e2, S.red);
  } else {
    double inner = 0.0;
    for (int e = t; e < I0 * R; e += 256) inner += A0[e] * M0[e];
    out = block_sum(inner, S.red);
  }
  return out;
}

__device__ double pass_dispatch(const BFit& f, const double* Ain, double* Mout, int resid, Smem& S) {
  if (f.dtype == 0) return bpass<double>(f, Ain, Mout, resid, S);
  return bpass<float>(f, Ain, Mout, resid, S);
}

// sum_{r,s} prod_n C_n[r,s] (= ||Y_hat||^2) from LDS Grams.
__device__ double yhat2(const BFit& f, const double (*Cs)[BR2], Smem& S) {
  const int R = f.R;
  double v = 0.0;
  for (int e = threadIdx.x; e < BR2; e += 256) {
    const int r = e & 7, q = e >> 3;
    if (r < R && q < R) v += Cs[0][r + q * R] * Cs[1][r + q * R] * Cs[2][r + q * R];
  }
  return block_sum(v, S.red);
}

// Grams of the stacked factors Ain into Cdst (LDS) and Cglob.
__device__ void grams(const BFit& f, const double* Ain, double (*Cdst)[BR2], double* Cglob) {
  const int t = threadIdx.x, R = f.R;
  sync_block();
  if (t < 3 * BR2) {
    const int n = t >> 6, e = t & 63, r = e & 7, q = e >> 3;
    if (r < R && q < R) {
      const int In = f.I[n];
      const double* An = Ain + aoff(f, n);
      double acc = 0.0;
      for (int i = 0; i < In; ++i) acc += An[i + (long long)r * In] * An[i + (long long)q * In];
      Cdst[n][r + q * R] = acc;
      Cglob[n * BR2 + r + q * R] = acc;
    }
  }
  sync_block();
}

__device__ double gamma_of(const double (*Cs)[BR2], int skip1, int skip2, int e) {
  double g = 1.0;
  for (int k = 0; k < 3; ++k)
    if (k != skip1 && k != skip2) g *= Cs[k][e];
  return g;
}

// Serial R x R work of one mode (R <= 8) by one thread: Gamma_n, Cholesky of
// Gamma_n + mu I, X_n = L^-T, Gt_n = X_n X_n^T, semidefinite-safe L of C_n.
// R x R work of mode n by one wave, lane (r, q) = (lane & 7, lane >> 3) holding
// entry (r, q): Gamma_n, the Cholesky factor L of Gamma_n + mu I (a
// non-positive pivot raises the singular flag), X_n = L^-T, Gt_n = X_n X_n^T,
// and the semidefinite-safe Cholesky factor L_n of C_n.  The factorisations
// are right-looking on the full symmetric matrix; the column and pivot of a
// step are broadcast with lane shuffles.
__device__ void rr_mode(const BFit& f, int n, double mu, Smem& S) {
  const int R = f.R, lane = threadIdx.x & 63, r = lane & 7, q = lane >> 3;
  const bool act = r < R && q < R;
  const int e = r + q * R;
  double g = 0.0;
  if (act) {
    g = gamma_of(S.Cs, n, -1, e);
    S.Gm[n][e] = g;
  }
  double h = g + ((r == q) ? mu : 0.0);
  for (int k = 0; k < R; ++k) {
    const double piv = __shfl(h, 9 * k);
    const double lrk = __shfl(h, r + 8 * k), lqk = __shfl(h, q + 8 * k);
    double d = 1.0;
    if (piv > 0.0) d = sqrt(piv);
    else if (lane == 0) S.flags[0] = 1;
    if (r > k && q > k) h -= (lrk / d) * (lqk / d);
    else if (q == k && r > k) h = lrk / d;
    else if (q == k && r == k) h = d;
  }
  // column q of L^-1 by forward substitution, one step per column of L
  double x = (r == q) ? 1.0 : 0.0;
  for (int k = 0; k < R; ++k) {
    const double lkk = __shfl(h, 9 * k);
    const double xkq = __shfl(x, k + 8 * q) / lkk;
    const double lrk = __shfl(h, r + 8 * k);
    if (r == k) x = xkq;
    else if (r > k) x -= lrk * xkq;
  }
  const double xt = __shfl(x, q + 8 * r);  // Li[q][r]
  double gt = 0.0;
  for (int k = 0; k < R; ++k) {
    const double a = __shfl(x, k + 8 * r), b = __shfl(x, k + 8 * q);
    if (k >= r && k >= q) gt += a * b;
  }
  if (act) {
    S.Xs[n][e] = xt;
    S.Gt[n][e] = gt;
  }
  // L L^T = C_n, a pivot below 64 u times its diagonal zeroing the column
  double c = act ? S.Cs[n][e] : 0.0;
  for (int k = 0; k < R; ++k) {
    const double piv = __shfl(c, 9 * k);
    const double lrk = __shfl(c, r + 8 * k), lqk = __shfl(c, q + 8 * k);
    const bool zero = !(piv > 64.0 * 2.220446049250313e-16 * S.Cs[n][k + k * R]);
    const double d = zero ? 0.0 : sqrt(piv);
    if (r > k && q > k) c -= zero ? 0.0 : (lrk / d) * (lqk / d);
    else if (q == k && r > k) c = zero ? 0.0 : lrk / d;
    else if (q == k && r == k) c = d;
  }
  if (act) S.Ls[n][e] = (q <= r) ? c : 0.0;
}

// Per-fit initial state: ||Y||^2, Grams, first tensor pass, err2, mu0.
__device__ void binit_body(const BFit& f, const BatchCfg& cfg, Smem& S) {
  const int t = threadIdx.x, R = f.R;
  FitState* st = f.st;
  // stacked copy of the caller's factors
  for (int n = 0; n < 3; ++n) {
    const long long o = aoff(f, n);
    for (int e = t; e < f.I[n] * R; e += 256) f.A[o + e] = f.Ain[n][e];
  }
  const long long J = (long long)f.I[0] * f.I[1] * f.I[2];
  double yy = 0.0;
  if (f.dtype == 0) {
    const double* y = static_cast<const double*>(f.Y);
    for (long long i = t; i < J; i += 256) yy += y[i] * y[i];
  } else {
    const float* y = static_cast<const float*>(f.Y);
    for (long long i = t; i < J; i += 256) yy += (double)y[i] * (double)y[i];
  }
  yy = block_sum(yy, S.red);
  grams(f, f.A, S.Cs, f.C);
  const int resid = (f.dtype == 0) || cfg.resid_switch < 0.0;
  const double pv = pass_dispatch(f, f.A, f.M, resid, S);
  const double err2 = resid ? pv : yy - 2.0 * pv + yhat2(f, S.Cs, S);
  if (t == 0) {
    double mu = f.mu0;
    if (!(mu > 0.0)) {
      double mx = 0.0;
      for (int n = 0; n < 3; ++n)
        for (int r = 0; r < R; ++r) {
          const double g = gamma_of(S.Cs, n, -1, r + r * R);
          mx = g > mx ? g : mx;
        }
      mu = cfg.tau * mx;
    }
    st->mu = mu;
    st->mu0 = mu;
    st->ynorm2 = yy;
    st->ynorm2_pass = yy;
    st->err2 = err2;
    st->eps = sqrt(err2 / yy);
    st->eps_prev = st->eps;
    st->iters = 0;
    st->accepted = 0;
    st->tol = cfg.tol;
    st->max_iters = cfg.max_iters;
    st->normalize = cfg.normalize;
    st->stop = (isfinite(err2) && mu > 0.0 && cfg.max_iters > 0) ? 0 : 1;
    st->reason = (isfinite(err2) && mu > 0.0) ? 1 : 3;
    st->singular = 0;
    st->resid = resid;
    st->resid_iters = 0;
    st->pad0 = 0;  // refresh pending
    st->mu_rule = cfg.mu_rule;
    st->nu = 2.0;
    st->t0_ticks = (long long)wall_clock64();
    st->t1_ticks = st->t0_ticks;
    if (st->stop) atomicAdd(cfg.nstopped, 1);
  }
}

__global__ __launch_bounds__(256) void k_binit(BFit* fits, int nfits, BatchCfg cfg) {
  __shared__ Smem S;
  const int fi = blockIdx.x;
  if (fi >= nfits) return;
  binit_body(fits[fi], cfg, S);
}

// One trial of an unfinished fit (returns at once for a stopped one).
__device__ void btrial_body(const BFit& f, const BatchCfg& cfg, Smem& S) {
  FitState* st = f.st;
  if (st->stop) return;
  const int t = threadIdx.x, lane = t & 63, R = f.R, R2 = R * R, N = 3;
  const int T = f.I[0] + f.I[1] + f.I[2];
  const int nt = 2 * R2;
  if (t < 8) S.flags[t] = 0;
  // residual-corrected pass requested at the previous trial: refresh M and err2
  int resid = st->resid;
  if (st->pad0) {
    const double e2 = pass_dispatch(f, f.A, f.M, 1, S);
    if (t == 0) {
      st->err2 = e2;
      st->eps = sqrt(e2 / st->ynorm2);
      st->pad0 = 0;
    }
  }
  const double mu = st->mu;
  sync_block();
  // Grams of the current factors (kept in the workspace)
  for (int e = t; e < 3 * BR2; e += 256) S.Cs[e >> 6][e & 63] = f.C[e];
  sync_block();
  // S1: R x R work per mode
  if (t < 192) rr_mode(f, t >> 6, mu, S);
  sync_block();
  // S2: gradient rows G, P = G Gt
  if (t < T) {
    int i;
    const int n = mode_of_row(f, t, &i);
    const int In = f.I[n];
    const long long o = aoff(f, n);
    // the row in registers: loops over the rank are unrolled to BR with guards
    double g[BR], a[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      a[r] = (r < R) ? f.A[o + i + (long long)r * In] : 0.0;
      g[r] = (r < R) ? f.M[o + i + (long long)r * In] : 0.0;
    }
    if (!resid)
#pragma unroll
      for (int r = 0; r < BR; ++r) {
        if (r < R) {
          double acc = 0.0;
#pragma unroll
          for (int s2 = 0; s2 < BR; ++s2)
            if (s2 < R) acc += a[s2] * S.Gm[n][s2 + r * R];
          g[r] -= acc;
        }
      }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      if (r < R) {
        double acc = 0.0;
#pragma unroll
        for (int s2 = 0; s2 < BR; ++s2)
          if (s2 < R) acc += g[s2] * S.Gt[n][s2 + r * R];
        f.G[o + i + (long long)r * In] = g[r];
        f.P[o + i + (long long)r * In] = acc;
      }
    }
  }
  sync_block();
  // w_n = vec(A_n^T P_n)
  if (t < 3 * BR2) {
    const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
    if (a < R && b < R) {
      const int In = f.I[n];
      const long long o = aoff(f, n);
      double acc = 0.0;
      for (int i = 0; i < In; ++i) acc += f.A[o + i + (long long)a * In] * f.P[o + i + (long long)b * In];
      S.w[n * R2 + a + b * R] = acc;
    }
  }
  sync_block();
  // S3: z_n = vec(L_n^T (sum_{m != n} Gamma_nm * W_m^T) X_n)
  {
    auto& rr = S.u.rr;
    if (t < 3 * BR2) {
      const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
      if (a < R && b < R) {
        double v = 0.0;
        for (int m = 0; m < N; ++m)
          if (m != n) v += gamma_of(S.Cs, n, m, a + b * R) * S.w[m * R2 + b + a * R];
        rr.V[n][a + b * R] = v;
      }
    }
    sync_block();
    if (t < 3 * BR2) {
      const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
      if (a < R && b < R) {
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += S.Ls[n][k + a * R] * rr.V[n][k + b * R];
        rr.T1[n][a + b * R] = acc;
      }
    }
    sync_block();
    if (t < 3 * BR2) {
      const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
      if (a < R && b < R) {
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += rr.T1[n][a + k * R] * S.Xs[n][k + b * R];
        S.z[n * R2 + a + b * R] = acc;
      }
    }
    sync_block();
  }
  // S4: trailing system (packed lower, rows 0..nt with the RHS as row nt) and B
  auto& Y = S.u.sys;
  for (int p = t; p < nt; p += 256)
    for (int q = 0; q <= p; ++q) Y.Sp[pidx(p, q)] = (p == q) ? 1.0 : 0.0;
  sync_block();
  for (int pr = 0; pr < 3; ++pr) {
    const int n = (pr == 0) ? 1 : 2, m = (pr == 2) ? 1 : 0;
    // Tb[(a + d R) R + i] = sum_j Gamma_nm[i,j] L_n[j,a] X_m[j,d]
    for (int e = t; e < R * R2; e += 256) {
      const int i = e % R, ad = e / R, a = ad % R, d = ad / R;
      double acc = 0.0;
      for (int j = 0; j < R; ++j) acc += gamma_of(S.Cs, n, m, i + j * R) * S.Ls[n][j + a * R] * S.Xs[m][j + d * R];
      Y.Tb[e] = acc;
    }
    sync_block();
    for (int e = t; e < R2 * R2; e += 256) {
      const int a = e % R, b = (e / R) % R, c = (e / R2) % R, d = e / (R2 * R);
      double acc = 0.0;
      for (int i = 0; i < R; ++i) acc += S.Xs[n][i + b * R] * S.Ls[m][i + c * R] * Y.Tb[(a + d * R) * R + i];
      const int p = (n - 1) * R2 + a + b * R;
      if (m == 0) Y.Bm[p][c + d * R] = acc;
      else Y.Sp[pidx(p, (m - 1) * R2 + c + d * R)] = acc;
    }
    sync_block();
  }
  // Schur update with block 1 (S_tt -= B B^T on the FP64 matrix cores, one
  // 16 x 16 lower tile per wave at a time) and the right-hand side row.
  // v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16] and B[l/16][l%16] of the
  // step and the result D[l/16 + 4v][l%16]; rows of B beyond nt only reach
  // outputs that are not stored, columns of B beyond R^2 are masked to zero.
  {
    const int w = t >> 6, li = lane & 15, lq = lane >> 4;
    const int nT = (nt + 15) >> 4, ntile = nT * (nT + 1) / 2, K4 = (R2 + 3) & ~3;
    for (int tile = w; tile < ntile; tile += 4) {
      int P = 0;
      while ((P + 1) * (P + 2) / 2 <= tile) ++P;
      const int Q = tile - P * (P + 1) / 2;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < K4; k0 += 4) {
        const int k = k0 + lq;
        const double a = (k < R2) ? Y.Bm[16 * P + li][k] : 0.0;
        const double b = (k < R2) ? Y.Bm[16 * Q + li][k] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pr = 16 * P + lq + 4 * v, qc = 16 * Q + li;
        if (pr < nt && qc <= pr) Y.Sp[pidx(pr, qc)] -= acc[v];
      }
    }
  }
  for (int p = t; p < nt; p += 256) {
    double acc = 0.0;
    for (int k = 0; k < R2; ++k) acc += Y.Bm[p][k] * S.z[k];
    Y.Sp[pidx(nt, p)] = S.z[R2 + p] - acc;
  }
  // S5: Cholesky of the trailing system; row nt becomes L^-1 z'.  One barrier
  // per column: step k updates the columns right of k from the unscaled
  // column k (every thread scales the entries it reads), and column k itself
  // is scaled in step k + 1, when nothing reads it any more.
  double dprev = 1.0;
  for (int k = 0; k < nt; ++k) {
    sync_block();
    const double dkk = Y.Sp[pidx(k, k)];
    double d = 1.0;
    if (dkk > 0.0) d = sqrt(dkk);
    else if (t == 0) S.flags[0] = 1;
    const double inv = 1.0 / d;
    if (k > 0) {
      for (int i = k + t; i <= nt; i += 256) Y.Sp[pidx(i, k - 1)] *= 1.0 / dprev;
      if (t == 0) Y.Sp[pidx(k - 1, k - 1)] = dprev;
    }
    // rows i in (k, nt], each row's columns j in (k, min(i, nt - 1)] split over
    // `js` threads (js = 256 / rows, at most 8), so no thread runs a long chain
    {
      const int rows = nt - k;
      const int js = rows >= 128 ? 2 : (rows >= 64 ? 4 : 8);
      const int ri = t / js, part = t - ri * js;
      for (int i = k + 1 + ri; i <= nt; i += 256 / js) {
        const double li = Y.Sp[pidx(i, k)] * inv;
        for (int j = k + 1 + part; j <= i && j < nt; j += js) Y.Sp[pidx(i, j)] -= li * (Y.Sp[pidx(j, k)] * inv);
      }
    }
    dprev = d;
  }
  sync_block();
  if (nt > 0) {
    for (int i = nt + t; i <= nt; i += 256) Y.Sp[pidx(i, nt - 1)] *= 1.0 / dprev;
    if (t == 0) Y.Sp[pidx(nt - 1, nt - 1)] = dprev;
  }
  sync_block();
  // backward substitution L^T y_t = v by wave 0 (rows lane and lane + 64)
  if (t < 64) {
    double v0 = (lane < nt) ? Y.Sp[pidx(nt, lane)] : 0.0;
    double v1 = (lane + 64 < nt) ? Y.Sp[pidx(nt, lane + 64)] : 0.0;
    for (int c = nt - 1; c >= 0; --c) {
      const double own = (c < 64) ? v0 : v1;
      const long long b = __double_as_longlong(own);
      const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), c & 63);
      const int hi = __builtin_amdgcn_readlane((int)(b >> 32), c & 63);
      const double yc = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo) / Y.Sp[pidx(c, c)];
      if (lane == 0) S.y[R2 + c] = yc;
      if (lane < c) v0 -= Y.Sp[pidx(c, lane)] * yc;
      if (lane + 64 < c) v1 -= Y.Sp[pidx(c, lane + 64)] * yc;
    }
  }
  sync_block();
  // y_1 = z_1 - B^T y_t
  if (t < R2) {
    double acc = 0.0;
    for (int p = 0; p < nt; ++p) acc += Y.Bm[p][t] * S.y[R2 + p];
    S.y[t] = S.z[t] - acc;
  }
  sync_block();
  // S6: u_n = w_n - vec(L_n Y_n X_n^T) (into v), f_n and Q_n = F_n Gt_n
  {
    auto& rr = S.u.rr;  // the system is no longer needed
    if (t < 3 * BR2) {
      const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
      if (a < R && b < R) {
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += S.Ls[n][a + k * R] * S.y[n * R2 + k + b * R];
        rr.T1[n][a + b * R] = acc;
      }
    }
    sync_block();
    if (t < 3 * BR2) {
      const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
      if (a < R && b < R) {
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += rr.T1[n][a + k * R] * S.Xs[n][b + k * R];
        S.v[n * R2 + a + b * R] = S.w[n * R2 + a + b * R] - acc;
      }
    }
    sync_block();
    if (t < 3 * BR2) {
      const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
      if (a < R && b < R) {
        double v = 0.0;
        for (int m = 0; m < N; ++m)
          if (m != n) v += gamma_of(S.Cs, n, m, a + b * R) * S.v[m * R2 + b + a * R];
        rr.V[n][a + b * R] = v;
      }
    }
    sync_block();
    if (t < 3 * BR2) {
      const int n = t >> 6, e = t & 63, a = e & 7, b = e >> 3;
      if (a < R && b < R) {
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += rr.V[n][a + k * R] * S.Gt[n][k + b * R];
        S.Qs[n][a + b * R] = acc;
      }
    }
    sync_block();
  }
  // S7: update rows A_c = A + P - A Q_n, gain-ratio denominator
  double den = 0.0;
  if (t < T) {
    int i;
    const int n = mode_of_row(f, t, &i);
    const int In = f.I[n];
    const long long o = aoff(f, n);
    double a[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) a[r] = (r < R) ? f.A[o + i + (long long)r * In] : 0.0;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      if (r < R) {
        double acc = 0.0;
#pragma unroll
        for (int s2 = 0; s2 < BR; ++s2)
          if (s2 < R) acc += a[s2] * S.Qs[n][s2 + r * R];
        const long long gi = o + i + (long long)r * In;
        const double da = f.P[gi] - acc;
        f.Ac[gi] = a[r] + da;
        den += da * (f.G[gi] + mu * da);
      }
    }
  }
  den = block_sum(den, S.red);
  // candidate Grams into LDS rr scratch and the workspace
  __shared__ double Cc[3][BR2];
  grams(f, f.Ac, Cc, f.Cc);
  // S8: tensor pass at the candidate
  const double pv = pass_dispatch(f, f.Ac, f.Mc, resid, S);
  double err2c;
  if (resid) {
    err2c = pv;
  } else {
    double yh = 0.0;
    for (int e = t; e < BR2; e += 256) {
      const int r = e & 7, q = e >> 3;
      if (r < R && q < R) yh += Cc[0][r + q * R] * Cc[1][r + q * R] * Cc[2][r + q * R];
    }
    yh = block_sum(yh, S.red);
    err2c = st->ynorm2_pass - 2.0 * pv + yh;
  }
  // S9: damping control, normalisation and commit
  __shared__ int accept_s;
  if (t == 0) {
    int accept = 0;
    const double rho = (st->err2 - err2c) / den;
    st->denom = den;
    st->rho = rho;
    st->err2_cand = err2c;
    st->iters += 1;
    if (resid) st->resid_iters += 1;
    // a non-positive pivot rejects the trial (mu grows), as in the single fit
    const int sing = S.flags[0] != 0;
    if (!sing && (!isfinite(err2c) || !isfinite(den))) {
      st->stop = 1;
      st->reason = 3;
    } else {
      if (!sing && err2c < st->err2) {
        accept = 1;
        st->accepted += 1;
        st->eps_prev = st->eps;
        st->err2 = err2c;
        st->eps = sqrt(err2c / st->ynorm2);
        const double t3 = 2.0 * rho - 1.0;
        double fct = 1.0 - t3 * t3 * t3;
        if (fct < 1.0 / 3.0) fct = 1.0 / 3.0;
        st->mu *= fct;
        st->nu = 2.0;
        if (fabs(st->eps_prev - st->eps) < st->tol) {
          st->stop = 1;
          st->reason = 0;
        } else if (!resid && cfg.resid_switch > 0.0 && fabs(st->eps_prev - st->eps) < cfg.resid_switch) {
          st->resid = 1;
          st->pad0 = 1;
        }
      } else if (st->mu_rule == 1) {
        st->mu *= st->nu;
        st->nu *= 2.0;
      } else {
        st->mu *= 2.0;
      }
      if (!st->stop && st->mu > 1e30) {
        st->stop = 1;
        st->reason = 2;
      }
      if (!st->stop && st->iters >= st->max_iters) {
        st->stop = 1;
        st->reason = 1;
      }
    }
    if (st->stop) {
      st->t1_ticks = (long long)wall_clock64();
      atomicAdd(cfg.nstopped, 1);
    }
    accept_s = accept;
  }
  sync_block();
  if (!accept_s) return;
  __shared__ double sc[3][BR];
  if (t < R) {
    double nr[3], lam = 1.0;
    bool ok = true;
    for (int n = 0; n < 3; ++n) {
      nr[n] = sqrt(Cc[n][t + t * R]);
      ok = ok && nr[n] > 0.0;
      lam *= nr[n];
    }
    for (int n = 0; n < 3; ++n) {
      double s2 = 1.0;
      if (ok) {
        if (st->normalize == 0) {
          s2 = pow(lam, 1.0 / 3.0) / nr[n];
        } else if (st->normalize == 1) {
          s2 = (n < 2) ? 1.0 / nr[n] : nr[0] * nr[1];
        }
      }
      sc[n][t] = s2;
    }
  }
  sync_block();
  if (t < T) {
    int i;
    const int n = mode_of_row(f, t, &i);
    const int In = f.I[n];
    const long long o = aoff(f, n);
    for (int r = 0; r < R; ++r) {
      double other = 1.0;
      for (int k = 0; k < 3; ++k)
        if (k != n) other *= sc[k][r];
      const long long gi = o + i + (long long)r * In;
      f.A[gi] = f.Ac[gi] * sc[n][r];
      f.M[gi] = f.Mc[gi] * other;
    }
  }
  if (t < 3 * BR2) {
    const int n = t >> 6, e = t & 63, r = e & 7, q = e >> 3;
    if (r < R && q < R) f.C[n * BR2 + r + q * R] = Cc[n][r + q * R] * sc[n][r] * sc[n][q];
  }
}

// One trial for every unfinished fit, one block per fit.
__global__ __launch_bounds__(256) void k_btrial(BFit* fits, int nfits, BatchCfg cfg) {
  __shared__ Smem S;
  const int fi = blockIdx.x;
  if (fi >= nfits) return;
  btrial_body(fits[fi], cfg, S);
}

// Copy the result factors back to the caller's buffers.
__device__ void bfinal_body(const BFit& f) {
  for (int n = 0; n < 3; ++n) {
    const long long o = aoff(f, n);
    for (int e = threadIdx.x; e < f.I[n] * f.R; e += 256) f.Ain[n][e] = f.A[o + e];
  }
}

__global__ __launch_bounds__(256) void k_bfinal(BFit* fits, int nfits) {
  const int fi = blockIdx.x;
  if (fi >= nfits) return;
  bfinal_body(fits[fi]);
}

// Persistent launch: each block takes the next fit from a queue (in the order
// given, largest first) and runs it from its initial state to its stop, then
// takes the next, so uneven fits share the CUs without a launch or a grid-wide
// step per trial.  Every block leaves once the queue is past the last fit;
// every fit runs at most max_iters trials.  copy_out = 0 leaves the caller's
// factors untouched (timing runs of the tuner).
__global__ __launch_bounds__(256) void k_bpersist(BFit* fits, int nfits, const int* order, int* queue,
                                                  BatchCfg cfg, int ntrials, int copy_out) {
  __shared__ Smem S;
  __shared__ int slot_s, stop_s;
  for (;;) {
    sync_block();
    if (threadIdx.x == 0) slot_s = atomicAdd(queue, 1);
    sync_block();
    const int slot = slot_s;
    if (slot >= nfits) return;
    const BFit f = fits[order[slot]];
    binit_body(f, cfg, S);
    for (int it = 0; it < ntrials; ++it) {
      sync_block();
      if (threadIdx.x == 0) stop_s = __hip_atomic_load(&f.st->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sync_block();
      if (stop_s) break;
      btrial_body(f, cfg, S);
    }
    sync_block();
    if (copy_out) bfinal_body(f);
  }
}

__global__ void k_bqueue_reset(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

}  // namespace

bool batched_supported(int order, const int64_t* dims, int R) {
  if (order != 3 || R < 1 || R > BR) return false;
  for (int n = 0; n < 3; ++n)
    if (dims[n] < 1 || dims[n] > BI) return false;
  return true;
}

size_t batched_fit_doubles(const int* I, int R) {
  const size_t TR = (size_t)(I[0] + I[1] + I[2]) * R;
  return 6 * TR + 2 * 3 * BR2;
}

hipError_t launch_batched_init(BFit* fits, int nfits, const BatchCfg& cfg, hipStream_t st) {
  k_binit<<<nfits, 256, 0, st>>>(fits, nfits, cfg);
  return hipGetLastError();
}

hipError_t launch_batched_trial(BFit* fits, int nfits, const BatchCfg& cfg, hipStream_t st) {
  k_btrial<<<nfits, 256, 0, st>>>(fits, nfits, cfg);
  return hipGetLastError();
}

hipError_t launch_batched_final(BFit* fits, int nfits, hipStream_t st) {
  k_bfinal<<<nfits, 256, 0, st>>>(fits, nfits);
  return hipGetLastError();
}

hipError_t launch_batched_persistent(BFit* fits, int nfits, const int* order, int* queue, const BatchCfg& cfg,
                                     int blocks, int ntrials, bool copy_out, hipStream_t st) {
  k_bqueue_reset<<<1, 64, 0, st>>>(queue);
  k_bpersist<<<blocks, 256, 0, st>>>(fits, nfits, order, queue, cfg, ntrials, copy_out ? 1 : 0);
  return hipGetLastError();
}

}  // namespace dgn
