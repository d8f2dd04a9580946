// Device-resident damping control of the fit (Algorithm 1, Section 4.5).
//
// One iteration is one trial step.  The residual of the candidate comes from
// the tensor pass at the candidate factors: either directly (sum of E^2 in
// the residual-corrected pass) or as ||Y||^2 - 2 <Y, Y_hat> + ||Y_hat||^2 with
// <Y, Y_hat> = sum(A_1 * M_1) and ||Y_hat||^2 = sum_{r,s} prod_n C_n[r,s].
// A trial is accepted iff the residual decreases; then mu <- mu max(1/3,
// 1 - (2 rho - 1)^3), else mu <- 2 mu (the rule as Section 4.5 prints it) or,
// with Nielsen's rule (the damping reference of Section 4.5), mu <- mu nu and
// nu <- 2 nu, nu returning to 2 on every acceptance.  Accepted factors are normalised; the
// stored MTTKRP (or gradient) columns and Gram matrices are rescaled with the
// same column scales, which leave Y_hat unchanged.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

// err2 of factors A with pass output M (mode 1 block) and Grams C.  With
// ipart, <A_1, M_1> is the sum of its nip pieces.  red: 32 doubles of shared
// memory; the two sums share one block reduction.
__device__ double err2_of(const Shape& s, const double* A, const double* M, const double* C,
                          int resid, const double* e2, double ynorm2_pass, double* red,
                          const double* ipart = nullptr, int nip = 0) {
  if (resid) return e2[0];
  const int R = s.R, R2 = R * R, I0 = s.I[0];
  // 16 independent loads per thread in flight: the operands are a few hundred KB
  const int n = ipart ? nip : I0 * R, bd = blockDim.x;
  double part[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int e = threadIdx.x;
  if (ipart) {
    for (; e + 7 * bd < n; e += 8 * bd)
#pragma unroll
      for (int q = 0; q < 8; ++q) part[q] += ipart[e + q * bd];
    for (; e < n; e += bd) part[0] += ipart[e];
  } else {
    for (; e + 7 * bd < n; e += 8 * bd)
#pragma unroll
      for (int q = 0; q < 8; ++q) part[q] += A[e + q * bd] * M[e + q * bd];
    for (; e < n; e += bd) part[0] += A[e] * M[e];
  }
  double inner = ((part[0] + part[1]) + (part[2] + part[3])) + ((part[4] + part[5]) + (part[6] + part[7]));
  // ||Y_hat||^2 = sum over (r, s) of prod_n C_n[r, s]; the loads of four entries in flight
  double yh = 0.0;
  for (int e0 = threadIdx.x; e0 < R2; e0 += 4 * bd) {
    double cv[4][kMaxOrder];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < kMaxOrder; ++k) {
        const int x = e0 + u * bd;
        cv[u][k] = (k < s.N && x < R2) ? C[(long long)k * R2 + x] : 1.0;
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double g = 1.0;
#pragma unroll
      for (int k = 0; k < kMaxOrder; ++k) g *= cv[u][k];
      if (e0 + u * bd < R2) yh += g;
    }
  }
  inner = wave_sum(inner);
  yh = wave_sum(yh);
  const int w = threadIdx.x / kWave, nw = bd / kWave;
  sync_block();
  if (threadIdx.x % kWave == 0) {
    red[w] = inner;
    red[16 + w] = yh;
  }
  sync_block();
  double si = 0.0, sy = 0.0;
  for (int i = 0; i < nw; ++i) {
    si += red[i];
    sy += red[16 + i];
  }
  sync_block();
  return ynorm2_pass - 2.0 * si + sy;
}

__global__ __launch_bounds__(256) void k_fit_init(Shape s, const double* A, const double* M,
                                                  const double* C, int resid, const double* e2,
                                                  double mu0, double tau, FitState* st, int cs) {
  __shared__ double red[32];
  const double err2 = err2_of(s, A, M, C, resid, e2, st->ynorm2_pass, red);
  if (threadIdx.x == 0) {
    const int R = s.R, R2 = R * R;
    double mu = mu0;
    if (!(mu0 > 0.0)) {
      double mx = 0.0;
      for (int n = 0; n < s.N; ++n)
        for (int r = 0; r < R; ++r) {
          double g = 1.0;
          for (int k = 0; k < s.N; ++k)
            if (k != n) g *= C[cs * ((long long)k * R2 + r + r * R)];
          mx = g > mx ? g : mx;
        }
      mu = tau * mx;
    }
    st->mu = mu;
    st->mu0 = mu;
    st->err2 = err2;
    st->eps = sqrt(err2 / st->ynorm2);
    st->eps_prev = st->eps;
    st->iters = 0;
    st->accepted = 0;
    st->stop = (isfinite(err2) && mu > 0.0) ? 0 : 1;
    st->reason = st->stop ? 3 : 1;
    st->commit_iter = -1;
    st->singular = 0;
    st->resid = resid;
    st->resid_iters = 0;
    st->nu = 2.0;
  }
}

// Residual of the current factors after a switch to the residual-corrected pass.
__global__ __launch_bounds__(256) void k_refresh(Shape s, const double* e2, FitState* st) {
  if (threadIdx.x == 0 && !st->stop) {
    st->err2 = e2[0];
    st->eps = sqrt(e2[0] / st->ynorm2);
    st->resid = 1;
  }
}

__global__ __launch_bounds__(256) void k_err2(Shape s, const double* A, const double* M,
                                              const double* C, int resid, const double* e2,
                                              const double* ynorm2_pass, double* out) {
  __shared__ double red[32];
  const double v = err2_of(s, A, M, C, resid, e2, ynorm2_pass[0], red);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ __launch_bounds__(256) void k_inner(Shape s, const double* A, const double* M,
                                               double* out) {
  __shared__ double red[32];
  double v = 0.0;
  for (int e = threadIdx.x; e < s.I[0] * s.R; e += blockDim.x) v += A[e] * M[e];
  v = block_sum(v, red);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ __launch_bounds__(256) void k_control(Shape s, const double* Ac, const double* Mc,
                                                 const double* Cc, int resid, const double* e2,
                                                 const double* scal, FitState* st, int trial, int cs,
                                                 const double* ipart, int nip) {
  __shared__ double red[32];
  __shared__ int accept_s;
  if (st->stop) return;
  const double err2c = err2_of(s, Ac, Mc, Cc, resid, e2, st->ynorm2_pass, red, ipart, nip);
  const int N = s.N, R = s.R, R2 = R * R;
  if (threadIdx.x == 0) {
    int accept = 0;
    const double denom = scal[0];
    st->denom = denom;
    st->danorm2 = scal[1];
    st->gnorm2 = scal[2];
    st->mnorm2 = scal[3];
    st->err2_cand = err2c;
    const double rho = (st->err2 - err2c) / denom;
    st->rho = rho;
    st->iters += 1;
    if (resid) st->resid_iters += 1;
    st->commit_iter = -1;
    // A non-positive pivot of (Gamma^(n) + mu I) or of the NR^2 system means the
    // damping is too small for the system to be positive definite in FP64: the
    // trial is rejected and mu grows as after a rise of the residual.
    const int sing = st->singular;
    st->singular = 0;
    if (!sing && (!isfinite(err2c) || !isfinite(denom))) {
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
        double f = 1.0 - t3 * t3 * t3;
        if (f < 1.0 / 3.0) f = 1.0 / 3.0;
        st->mu *= f;
        st->nu = 2.0;
        st->commit_iter = trial;
        if (fabs(st->eps_prev - st->eps) < st->tol) {
          st->stop = 1;
          st->reason = 0;
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
    accept_s = accept;
  }
  sync_block();
  // column scales of the normalisation (norms from the candidate Grams), one column per thread
  const int r = threadIdx.x;
  if (accept_s && r < R) {
    double nr[kMaxOrder];
    double lam = 1.0;
    bool ok = true;
    for (int n = 0; n < N; ++n) {
      nr[n] = sqrt(Cc[cs * ((long long)n * R2 + r + r * R)]);
      ok = ok && nr[n] > 0.0;
      lam *= nr[n];
    }
    const int mode = st->normalize;
    for (int n = 0; n < N; ++n) {
      double sc = 1.0;
      if (ok) {
        if (mode == 0) {
          sc = pow(lam, 1.0 / N) / nr[n];
        } else if (mode == 1) {
          if (n < N - 1) {
            sc = 1.0 / nr[n];
          } else {
            sc = 1.0;
            for (int k = 0; k < N - 1; ++k) sc *= nr[k];
          }
        }
      }
      st->scale[n * kMaxRank + r] = sc;
    }
  }
}

// Apply an accepted trial: A = Ac diag(s_n), M = Mc diag(prod_{k != n} s_k), C = s C s.
// cs = 2 for interleaved complex arrays (the scales are real).
__global__ __launch_bounds__(256) void k_commit(Shape s, double* A, const double* Ac, double* M,
                                                const double* Mc, double* C, const double* Cc,
                                                const FitState* st, int trial, int cs) {
  if (st->commit_iter != trial) return;
  const int n = blockIdx.x, c = blockIdx.y, R = s.R, R2 = R * R, In = s.I[n], N = s.N;
  const double* sc = st->scale;
  const long long base = (long long)s.off[n] * R;
  if (cs == 1) {
    // every load of the thread issued before the stores
    constexpr int NE = 64 * kMaxRank / 256;
    double av[NE], mv[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = threadIdx.x + 256 * k, ii = e & 63, r = e >> 6, i = c * 64 + ii;
      const bool ok = e < 64 * R && i < In;
      const long long gi = base + i + (long long)r * In;
      av[k] = ok ? Ac[gi] : 0.0;
      mv[k] = ok ? Mc[gi] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = threadIdx.x + 256 * k, ii = e & 63, r = e >> 6, i = c * 64 + ii;
      if (e < 64 * R && i < In) {
        const long long gi = base + i + (long long)r * In;
        double other = 1.0;
        for (int m = 0; m < N; ++m)
          if (m != n) other *= sc[m * kMaxRank + r];
        A[gi] = av[k] * sc[n * kMaxRank + r];
        M[gi] = mv[k] * other;
      }
    }
  } else {
    for (int e = threadIdx.x; e < 64 * R; e += 256) {
      const int ii = e & 63, r = e >> 6;
      const int i = c * 64 + ii;
      if (i >= In) continue;
      const long long gi = base + i + (long long)r * In;
      double other = 1.0;
      for (int k = 0; k < N; ++k)
        if (k != n) other *= sc[k * kMaxRank + r];
      for (int h = 0; h < cs; ++h) {
        A[cs * gi + h] = Ac[cs * gi + h] * sc[n * kMaxRank + r];
        M[cs * gi + h] = Mc[cs * gi + h] * other;
      }
    }
  }
  if (c == 0) {
    for (int q = (int)(threadIdx.x >> 6); q < R; q += 4)
      for (int r = (int)(threadIdx.x & 63); r < R; r += 64) {
        const long long e = (long long)n * R2 + r + q * R;
        for (int h = 0; h < cs; ++h)
          C[cs * e + h] = Cc[cs * e + h] * sc[n * kMaxRank + r] * sc[n * kMaxRank + q];
      }
  }
}

}  // namespace

hipError_t launch_fit_init(const Shape& s, const double* A, const double* M, const double* C,
                           bool resid, const double* e2, double mu0, double tau, FitState* state,
                           hipStream_t st, int cs) {
  k_fit_init<<<1, 256, 0, st>>>(s, A, M, C, resid ? 1 : 0, e2, mu0, tau, state, cs);
  return hipGetLastError();
}

hipError_t launch_refresh(const Shape& s, const double* e2, FitState* state, hipStream_t st) {
  k_refresh<<<1, 64, 0, st>>>(s, e2, state);
  return hipGetLastError();
}

hipError_t launch_err2(const Shape& s, const double* A, const double* M, const double* C, bool resid,
                       const double* e2, const double* ynorm2_pass, double* out, hipStream_t st) {
  k_err2<<<1, 256, 0, st>>>(s, A, M, C, resid ? 1 : 0, e2, ynorm2_pass, out);
  return hipGetLastError();
}

hipError_t launch_inner(const Shape& s, const double* A, const double* M, double* out, hipStream_t st) {
  k_inner<<<1, 256, 0, st>>>(s, A, M, out);
  return hipGetLastError();
}

hipError_t launch_control(const Shape& s, const double* Ac, const double* Mc, const double* Cc,
                          bool resid, const double* e2, const double* scal, FitState* state,
                          int trial, hipStream_t st, int cs, const double* ipart, int nip) {
  k_control<<<1, 256, 0, st>>>(s, Ac, Mc, Cc, resid ? 1 : 0, e2, scal, state, trial, cs, ipart, nip);
  return hipGetLastError();
}

hipError_t launch_commit(const Shape& s, double* A, const double* Ac, double* M, const double* Mc,
                         double* C, const double* Cc, const FitState* state, int trial,
                         hipStream_t st, int cs) {
  k_commit<<<dim3(s.N, row_chunks(s)), 256, 0, st>>>(s, A, Ac, M, Mc, C, Cc, state, trial, cs);
  return hipGetLastError();
}

}  // namespace dgn
