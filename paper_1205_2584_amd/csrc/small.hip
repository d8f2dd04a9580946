// FP64 kernels on the R x R objects and the factor rows of the fast step.
//
// Notation (Theorem 4.1 and Lemma 4.4):  C_n = A_n^T A_n, Gamma_n and
// Gamma_nm the Hadamard products of the C_k over k != n (k != n, m),
// Gt_n = (Gamma_n + mu I)^-1, G_n = Y_(n) KR - A_n Gamma_n (gradient block),
// P_n = G_n Gt_n (the block of G~_mu g), w_n = vec(A_n^T P_n).
//
// The NR^2 system is solved in the symmetric positive definite form
//   S = I + W^T K W,   W = blkdiag(X_n (x) L_n),  X_n X_n^T = Gt_n,  L_n L_n^T = C_n,
// so that Psi_mu = W W^T and f = K (I + Psi K)^-1 w = K (w - W S^-1 W^T K w).
// These kernels build X_n, L_n, z = W^T K w, and after the solve
// u = w - W y, f = K u, Q_n = F_n Gt_n and the update A_n + P_n - A_n Q_n.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

constexpr int LD = kMaxRank + 1;

// Loop over the R x R positions (r, q), R <= 64, without integer division:
// thread t takes r = t mod 2^sh and q = t / 2^sh + s blockDim / 2^sh, with
// 2^sh the smallest of 16, 32, 64 that covers R (declare RR_SHIFT first).
__device__ __forceinline__ int rr_shift_of(int R) { return R <= 16 ? 4 : (R <= 32 ? 5 : 6); }
#define RR_SHIFT const int rr_sh = rr_shift_of(R)
#define FOR_RR(r, q)                                                              \
  for (int q = (int)(threadIdx.x >> rr_sh); q < R; q += (int)(blockDim.x >> rr_sh)) \
    for (int r = (int)(threadIdx.x & ((1 << rr_sh) - 1)); r < R; r += (1 << rr_sh))

// FOR_RR for staging: the values of up to four q-steps of the thread are
// produced first (their loads in flight together), then put stores them.
// get(r, q) is also called for q = R - 1 in place of positions beyond R.
template <typename Get, typename Put>
__device__ __forceinline__ void for_rr_staged(int R, int sh, Get get, Put put) {
  const int r = (int)(threadIdx.x & ((1 << sh) - 1)), qs = (int)(blockDim.x >> sh);
  if (r >= R) return;
  for (int qb = (int)(threadIdx.x >> sh); qb < R; qb += 4 * qs) {
    decltype(get(0, 0)) v[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int q = qb + it * qs;
      v[it] = get(r, q < R ? q : R - 1);
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int q = qb + it * qs;
      if (q < R) put(r, q, v[it]);
    }
  }
}

struct d2 {
  double x, y;
};
struct d3 {
  double x, y, z;
};

// C_k[e] for every k < N (1 beyond N), loaded together.
__device__ __forceinline__ void load_c(const double* C, int N, int R2, int e, double (&cv)[kMaxOrder]) {
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) cv[k] = (k < N) ? C[(long long)k * R2 + e] : 1.0;
}

// prod_{k != s1, s2} cv[k] (an entry of Gamma_n or Gamma_nm), multiplied in the order of k.
__device__ __forceinline__ double prod_except(const double (&cv)[kMaxOrder], int s1, int s2) {
  double g = 1.0;
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) g *= (k == s1 || k == s2) ? 1.0 : cv[k];
  return g;
}

// Stage rows r0..r0+63 of the column-major In x R block src into S[ii][r]
// (zero outside), with every load of the thread issued before the LDS stores.
// Returns nothing; optional square-sum of the staged values through *sq.
__device__ __forceinline__ void stage_rows(double (*S)[LD], const double* src, int In, int r0, int R,
                                           double* sq = nullptr) {
  double v[16];
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, ii = e & 63, r = e >> 6;
    v[s2] = (r < R && r0 + ii < In) ? src[r0 + ii + (long long)r * In] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, ii = e & 63, r = e >> 6;
    if (r < R) S[ii][r] = v[s2];
    acc += v[s2] * v[s2];
  }
  if (sq) *sq += acc;
}

// Cholesky of the R x R matrix H (lower, in place) with 256 threads.
// mode 0: a non-positive pivot sets *bad.  mode 1 (semidefinite): a pivot
// below 64 u times the original diagonal zeroes the column.
__device__ void chol_lds(double (*H)[LD], int R, int mode, int* bad, double* lk) {
  const int t = threadIdx.x;
  for (int k = 0; k < R; ++k) {
    sync_block();
    const double dkk = H[k][k];
    double d = 1.0, inv = 1.0;
    bool zero = false;
    if (mode == 0) {
      if (!(dkk > 0.0)) {
        if (t == 0) *bad = 1;
      } else {
        d = sqrt(dkk);
        inv = 1.0 / d;
      }
    } else {
      const double ref = lk[64 + k];
      if (!(dkk > 64.0 * 2.220446049250313e-16 * ref)) {
        zero = true;
      } else {
        d = sqrt(dkk);
        inv = 1.0 / d;
      }
    }
    for (int i = k + t; i < R; i += blockDim.x) lk[i] = zero ? 0.0 : ((i == k) ? d : H[i][k] * inv);
    sync_block();
    for (int j = k + 1 + (int)(t >> 6); j < R; j += (int)(blockDim.x >> 6)) {
      const int i = t & 63;
      if (i >= j && i < R) H[i][j] -= lk[i] * lk[j];
    }
    for (int i = k + t; i < R; i += blockDim.x) H[i][k] = lk[i];
  }
  sync_block();
  RR_SHIFT;
  FOR_RR(i, j) {
    if (j > i) H[i][j] = 0.0;
  }
  sync_block();
}

// Gram partials of 64-row chunks: part[(n * chunks + c) * stride + (r + s R)].
__global__ __launch_bounds__(256) void k_gram_part(Shape s, const double* A, double* part,
                                                   int chunks, int stride, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double As[64][LD];
  const int n = blockIdx.x, c = blockIdx.y, R = s.R, In = s.I[n];
  RR_SHIFT;
  const int r0 = c * 64;
  double* out = part + ((long long)n * chunks + c) * stride;
  const double* An = A + (long long)s.off[n] * R;
  stage_rows(As, An, In, r0, R);
  sync_block();
  FOR_RR(r, q) {
    const int e = r + q * R;
    double acc = 0.0;
    for (int i = 0; i < 64; ++i) acc += As[i][r] * As[i][q];
    out[e] = acc;
  }
}

// out[n * R2 + x] = sum_c part[(n * chunks + c) * stride + x], x < R2, for the
// N blocks n < N.  With scal != nullptr, block N sums the two per-row scalars
// at offsets R2, R2 + 1 of every partial over all modes into scal[0], scal[1].
__global__ void k_rows_reduce(const double* part, int N, int chunks, int stride, int R2, double* out,
                              double* scal, const int* stop) {
  if (stopped(stop)) return;
  const int n = blockIdx.x;
  if (n == N) {
    if (threadIdx.x < 2) {
      double acc = 0.0;
      for (int m = 0; m < N; ++m)
        for (int c = 0; c < chunks; ++c) acc += part[((long long)m * chunks + c) * stride + R2 + threadIdx.x];
      scal[threadIdx.x] = acc;
    }
    return;
  }
  for (int x = threadIdx.x; x < R2; x += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += part[((long long)n * chunks + c) * stride + x];
    out[(long long)n * R2 + x] = acc;
  }
}

// Per mode n: Gamma_n, Cholesky of Gamma_n + mu I, its inverse factor
// X_n = L^-T, Gt_n = X_n X_n^T, and the (semidefinite-safe) Cholesky L_n of C_n.
__global__ __launch_bounds__(256) void k_gamma(Shape s, const double* C, double mu_host,
                                               const FitState* state, double* Gam, double* Gt,
                                               double* X, double* Lc, int* bad, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double H[64][LD];
  __shared__ double Li[64][LD];
  __shared__ double lk[128];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  RR_SHIFT;
  if (blockIdx.y == 1) {
    // the (semidefinite-safe) Cholesky L_n of C_n, in parallel with the damped inverse
    for_rr_staged(
        R, rr_sh, [&](int r, int q) { return C[(long long)n * R2 + r + q * R]; },
        [&](int r, int q, double v) { H[r][q] = v; });
    for (int r = t; r < R; r += 256) lk[64 + r] = C[(long long)n * R2 + r + r * R];
    chol_lds(H, R, 1, bad, lk);
    FOR_RR(r, q) {
      const int e = r + q * R;
      Lc[(long long)n * R2 + e] = H[r][q];
    }
    return;
  }
  const double mu = state ? state->mu : mu_host;
  for_rr_staged(
      R, rr_sh,
      [&](int r, int q) {
        double cv[kMaxOrder];
        load_c(C, N, R2, r + q * R, cv);
        return prod_except(cv, n, -1);
      },
      [&](int r, int q, double g) {
        Gam[(long long)n * R2 + r + q * R] = g;
        H[r][q] = g + (r == q ? mu : 0.0);
      });
  chol_lds(H, R, 0, bad, lk);
  // Li = L^-1, one column per thread (forward substitution on the identity)
  if (t < R) lk[t] = 1.0 / H[t][t];
  sync_block();
  for (int j = t; j < 64; j += 256) {
    if (j < R) {
      Li[j][j] = lk[j];
      for (int i = j + 1; i < R; ++i) {
        double acc = 0.0;
        for (int k = j; k < i; ++k) acc += H[i][k] * Li[k][j];
        Li[i][j] = -acc * lk[i];
      }
      for (int i = 0; i < j; ++i) Li[i][j] = 0.0;
    }
  }
  sync_block();
  FOR_RR(r, q) {
    const int e = r + q * R;
    // X = Li^T (upper triangular), Gt = Li^T Li
    X[(long long)n * R2 + e] = Li[q][r];
    const int k0 = r > q ? r : q;
    double acc = 0.0;
    for (int k = k0; k < R; ++k) acc += Li[k][r] * Li[k][q];
    Gt[(long long)n * R2 + e] = acc;
  }
}

// Rows of mode n, chunk c: G = M - A Gamma (or M itself when it already is the
// gradient), P = G Gt, partial w = A^T P, partial ||G||^2 and ||M||^2.
__global__ __launch_bounds__(256) void k_pw(Shape s, const double* A, const double* M, int resid,
                                            const double* Gam, const double* Gt, double* Gout,
                                            double* Pout, double* part, int chunks, int stride,
                                            const int* stop) {
  if (stopped(stop)) return;
  __shared__ double As[64][LD];
  __shared__ double Gs[64][LD];
  __shared__ double Ps[64][LD];
  __shared__ double Gm[64][LD];
  __shared__ double red[16];
  const int n = blockIdx.x, c = blockIdx.y, R = s.R, R2 = R * R, In = s.I[n], t = threadIdx.x;
  RR_SHIFT;
  const int r0 = c * 64;
  double* out = part + ((long long)n * chunks + c) * stride;
  if (r0 >= In) {
    for (int e = t; e < R2 + 4; e += 256) out[e] = 0.0;
    return;
  }
  const long long base = (long long)s.off[n] * R;
  const double* G0 = (resid ? Gt : Gam) + (long long)n * R2;
  for_rr_staged(
      R, rr_sh, [&](int r, int q) { return G0[r + q * R]; }, [&](int r, int q, double v) { Gm[r][q] = v; });
  double m2 = 0.0;
  stage_rows(As, A + base, In, r0, R);
  stage_rows(Gs, M + base, In, r0, R, &m2);
  sync_block();
  if (!resid) {
    // G = M - A Gamma
    for (int e = t; e < 64 * R; e += 256) {
      const int ii = e & 63, r = e >> 6;
      double acc = 0.0;
      for (int k = 0; k < R; ++k) acc += As[ii][k] * Gm[k][r];
      Ps[ii][r] = Gs[ii][r] - acc;
    }
    sync_block();
    for (int e = t; e < 64 * R; e += 256) {
      const int ii = e & 63, r = e >> 6;
      Gs[ii][r] = Ps[ii][r];
    }
    sync_block();
    for_rr_staged(
        R, rr_sh, [&](int r, int q) { return Gt[(long long)n * R2 + r + q * R]; },
        [&](int r, int q, double v) { Gm[r][q] = v; });
    sync_block();
  }
  double g2 = 0.0;
  for (int e = t; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Gs[ii][k] * Gm[k][r];
    Ps[ii][r] = acc;
    if (r0 + ii < In) {
      const long long gi = base + r0 + ii + (long long)r * In;
      Gout[gi] = Gs[ii][r];
      Pout[gi] = acc;
      g2 += Gs[ii][r] * Gs[ii][r];
    }
  }
  sync_block();
  FOR_RR(a, b) {
    const int e = a + b * R;
    double acc = 0.0;
    for (int i = 0; i < 64; ++i) acc += As[i][a] * Ps[i][b];
    out[e] = acc;
  }
  g2 = block_sum(g2, red);
  m2 = block_sum(m2, red);
  if (t == 0) {
    out[R2 + 0] = g2;
    out[R2 + 1] = m2;
    out[R2 + 2] = 0.0;
    out[R2 + 3] = 0.0;
  }
}

// w_n = sum over row chunks of the partial A_n^T P_n; block 0 also reduces
// ||G||^2 and ||M||^2 into scal[2], scal[3].
__global__ __launch_bounds__(256) void k_wred(Shape s, const double* part, int chunks, int stride,
                                              double* w, double* scal, const int* stop) {
  if (stopped(stop)) return;
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  for (int e = t; e < R2; e += 256) {
    const double* p0 = part + (long long)n * chunks * stride + e;
    double a0 = 0.0, a1 = 0.0;
    int c = 0;
    for (; c + 1 < chunks; c += 2) {
      a0 += p0[(long long)c * stride];
      a1 += p0[(long long)(c + 1) * stride];
    }
    if (c < chunks) a0 += p0[(long long)c * stride];
    w[(long long)n * R2 + e] = a0 + a1;
  }
  if (n == 0 && t < 2) {
    double acc = 0.0;
    for (int m = 0; m < N; ++m)
      for (int c = 0; c < chunks; ++c) acc += part[((long long)m * chunks + c) * stride + R2 + t];
    scal[2 + t] = acc;
  }
}

// Per mode n: V = sum_{m != n} Gamma_nm * W_m^T and z_n = vec(L_n^T V X_n) (= (W^T K w)_n).
__global__ __launch_bounds__(256) void k_z(Shape s, const double* C, const double* w,
                                           const double* X, const double* Lc, double* z,
                                           const int* stop) {
  if (stopped(stop)) return;
  __shared__ double V[64][LD];
  __shared__ double Ls[64][LD];
  __shared__ double Xs[64][LD];
  __shared__ double Tm[64][LD];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N;
  RR_SHIFT;
  for_rr_staged(
      R, rr_sh,
      [&](int a, int b) {
        const int e = a + b * R;
        double cv[kMaxOrder], wv[kMaxOrder];
        load_c(C, N, R2, e, cv);
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) wv[m] = (m < N && m != n) ? w[(long long)m * R2 + b + a * R] : 0.0;
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m)
          if (m < N && m != n) v += prod_except(cv, n, m) * wv[m];
        return d3{v, Lc[(long long)n * R2 + e], X[(long long)n * R2 + e]};
      },
      [&](int a, int b, d3 v) {
        V[a][b] = v.x;
        Ls[a][b] = v.y;
        Xs[a][b] = v.z;
      });
  sync_block();
  FOR_RR(a, b) {
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Ls[k][a] * V[k][b];
    Tm[a][b] = acc;
  }
  sync_block();
  FOR_RR(a, b) {
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Tm[a][k] * Xs[k][b];
    z[(long long)n * R2 + a + b * R] = acc;
  }
}

// T_nm[(a + d R) * R + i] = sum_j Gamma_nm[i, j] L_n[j, a] X_m[j, d] for n != m.
// Grid: (N * N pairs, R values of d).
__global__ __launch_bounds__(256) void k_tnm(Shape s, const double* C, const double* X,
                                             const double* Lc, double* Tnm, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Gs[64][LD];
  __shared__ double Ls[64][LD];
  __shared__ double xd[64];
  const int pair = blockIdx.x, d = blockIdx.y, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  RR_SHIFT;
  const int n = pair / N, m = pair % N;
  if (n == m) return;
  for_rr_staged(
      R, rr_sh,
      [&](int i, int j) {
        const int e = i + j * R;
        double cv[kMaxOrder];
        load_c(C, N, R2, e, cv);
        return d2{prod_except(cv, n, m), Lc[(long long)n * R2 + e]};
      },
      [&](int i, int j, d2 v) {
        Gs[i][j] = v.x;
        Ls[i][j] = v.y;
      });
  for (int j = t; j < R; j += 256) xd[j] = X[(long long)m * R2 + j + d * R];
  sync_block();
  double* out = Tnm + (long long)pair * R * R2;
  FOR_RR(i, a) {
    const int e = i + a * R;
    double acc = 0.0;
    for (int j = 0; j < R; ++j) acc += Gs[i][j] * Ls[j][a] * xd[j];
    out[((long long)a + (long long)d * R) * R + i] = acc;
  }
}

// u_n = w_n - vec(L_n Y_n X_n^T), Y_n = unvec(y_n).
__global__ __launch_bounds__(256) void k_u(Shape s, const double* w, const double* y,
                                           const double* X, const double* Lc, double* u,
                                           const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Ys[64][LD];
  __shared__ double Tm[64][LD];
  __shared__ double Ls[64][LD];
  __shared__ double Xs[64][LD];
  const int n = blockIdx.x, R = s.R, R2 = R * R;
  RR_SHIFT;
  for_rr_staged(
      R, rr_sh,
      [&](int r, int q) {
        const long long e = (long long)n * R2 + r + q * R;
        return d3{y[e], Lc[e], X[e]};
      },
      [&](int r, int q, d3 v) {
        Ys[r][q] = v.x;
        Ls[r][q] = v.y;
        Xs[r][q] = v.z;
      });
  sync_block();
  FOR_RR(a, b) {
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Ls[a][k] * Ys[k][b];
    Tm[a][b] = acc;
  }
  sync_block();
  FOR_RR(a, b) {
    const int e = a + b * R;
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Tm[a][k] * Xs[b][k];
    u[(long long)n * R2 + e] = w[(long long)n * R2 + e] - acc;
  }
}

// f_n = vec(sum_{m != n} Gamma_nm * U_m^T) (= (K u)_n), Q_n = F_n Gt_n.
__global__ __launch_bounds__(256) void k_fq(Shape s, const double* C, const double* u,
                                            const double* Gt, double* f, double* Q,
                                            const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Fs[64][LD];
  __shared__ double Gs[64][LD];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N;
  RR_SHIFT;
  for_rr_staged(
      R, rr_sh,
      [&](int a, int b) {
        const int e = a + b * R;
        double cv[kMaxOrder], uv[kMaxOrder];
        load_c(C, N, R2, e, cv);
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) uv[m] = (m < N && m != n) ? u[(long long)m * R2 + b + a * R] : 0.0;
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m)
          if (m < N && m != n) v += prod_except(cv, n, m) * uv[m];
        return d2{Gt[(long long)n * R2 + e], v};
      },
      [&](int a, int b, d2 v) {
        Gs[a][b] = v.x;
        f[(long long)n * R2 + a + b * R] = v.y;
        Fs[a][b] = v.y;
      });
  sync_block();
  FOR_RR(a, b) {
    const int e = a + b * R;
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Fs[a][k] * Gs[k][b];
    Q[(long long)n * R2 + e] = acc;
  }
}

// A_c = A + P - A Q_n on the rows of (mode n, chunk c).  Partials: Gram of A_c,
// sum da (g + mu da) and sum da^2.
__global__ __launch_bounds__(256) void k_update(Shape s, const double* A, const double* P,
                                                const double* G, const double* Q, double mu_host,
                                                const FitState* state, double* Ac, double* part,
                                                int chunks, int stride, double* da_out, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double As[64][LD];
  __shared__ double Qs[64][LD];
  __shared__ double Cs[64][LD];
  __shared__ double red[16];
  const int n = blockIdx.x, c = blockIdx.y, R = s.R, R2 = R * R, In = s.I[n], t = threadIdx.x;
  RR_SHIFT;
  const int r0 = c * 64;
  double* out = part + ((long long)n * chunks + c) * stride;
  if (r0 >= In) {
    for (int e = t; e < R2 + 4; e += 256) out[e] = 0.0;
    return;
  }
  const double mu = state ? state->mu : mu_host;
  const long long base = (long long)s.off[n] * R;
  for_rr_staged(
      R, rr_sh, [&](int r, int q) { return Q[(long long)n * R2 + r + q * R]; },
      [&](int r, int q, double v) { Qs[r][q] = v; });
  stage_rows(As, A + base, In, r0, R);
  sync_block();
  double den = 0.0, da2 = 0.0;
  for (int e = t; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    double v = 0.0;
    if (r0 + ii < In) {
      const long long gi = base + r0 + ii + (long long)r * In;
      double acc = 0.0;
      for (int k = 0; k < R; ++k) acc += As[ii][k] * Qs[k][r];
      const double da = P[gi] - acc;
      v = As[ii][r] + da;
      Ac[gi] = v;
      if (da_out) da_out[gi] = da;
      den += da * (G[gi] + mu * da);
      da2 += da * da;
    }
    Cs[ii][r] = v;
  }
  sync_block();
  FOR_RR(r, q) {
    const int e = r + q * R;
    double acc = 0.0;
    for (int i = 0; i < 64; ++i) acc += Cs[i][r] * Cs[i][q];
    out[e] = acc;
  }
  den = block_sum(den, red);
  da2 = block_sum(da2, red);
  if (t == 0) {
    out[R2 + 0] = den;
    out[R2 + 1] = da2;
    out[R2 + 2] = 0.0;
    out[R2 + 3] = 0.0;
  }
}

// ALS update of mode n (eq. ALS): A_n = M_n Gt_n with Gt_n = Gamma^(n)^-1
// (symmetric), one thread per entry of the column-major I_n x R block.
__global__ __launch_bounds__(256) void k_als_rows(Shape s, int n, const double* M, const double* Gt, double* A) {
  __shared__ double Gs[kMaxRank * kMaxRank];
  const int R = s.R, R2 = R * R, In = s.I[n], t = threadIdx.x;
  for (int e = t; e < R2; e += 256) Gs[e] = Gt[(long long)n * R2 + e];
  sync_block();
  const double* Mn = M + (long long)s.off[n] * R;
  double* An = A + (long long)s.off[n] * R;
  const long long total = (long long)In * R;
  for (long long e = blockIdx.x * 256LL + t; e < total; e += (long long)gridDim.x * 256) {
    const int i = (int)(e % In), r = (int)(e / In);
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Mn[i + (long long)k * In] * Gs[k + r * R];
    An[e] = acc;
  }
}

}  // namespace

int row_chunks(const Shape& s) { return (s.maxI + 63) / 64; }

static inline int part_stride(const Shape& s) { return s.R * s.R + 4; }

hipError_t launch_gram(const Shape& s, const double* A, const SmallBuffers& b, double* Cout,
                       const int* stop, hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride(s);
  k_gram_part<<<dim3(s.N, ch), 256, 0, st>>>(s, A, b.rowpart, ch, stride, stop);
  k_rows_reduce<<<s.N, 256, 0, st>>>(b.rowpart, s.N, ch, stride, s.R * s.R, Cout, nullptr, stop);
  return hipGetLastError();
}

hipError_t launch_gamma(const Shape& s, const double* C, double mu_host, const FitState* state,
                        const SmallBuffers& b, int* singular, const int* stop, hipStream_t st) {
  k_gamma<<<dim3(s.N, 2), 256, 0, st>>>(s, C, mu_host, state, b.Gam, b.Gt, b.X, b.Lc, singular, stop);
  return hipGetLastError();
}

hipError_t launch_pw(const Shape& s, const double* A, const double* M, bool resid,
                     const SmallBuffers& b, const int* stop, hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride(s);
  k_pw<<<dim3(s.N, ch), 256, 0, st>>>(s, A, M, resid ? 1 : 0, b.Gam, b.Gt, b.G, b.P, b.wpart, ch,
                                       stride, stop);
  return hipGetLastError();
}

hipError_t launch_wz(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride(s);
  k_wred<<<s.N, 256, 0, st>>>(s, b.wpart, ch, stride, b.w, b.scal, stop);
  k_z<<<s.N, 256, 0, st>>>(s, b.C, b.w, b.X, b.Lc, b.z, stop);
  return hipGetLastError();
}

hipError_t launch_tnm(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st) {
  k_tnm<<<dim3(s.N * s.N, s.R), 256, 0, st>>>(s, b.C, b.X, b.Lc, b.Tnm, stop);
  return hipGetLastError();
}

hipError_t launch_u(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st) {
  k_u<<<s.N, 256, 0, st>>>(s, b.w, b.y, b.X, b.Lc, b.u, stop);
  return hipGetLastError();
}

hipError_t launch_fq(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st) {
  k_fq<<<s.N, 256, 0, st>>>(s, b.C, b.u, b.Gt, b.f, b.Q, stop);
  return hipGetLastError();
}

hipError_t launch_update(const Shape& s, const double* A, double* Ac, const SmallBuffers& b,
                         double mu_host, const FitState* state, const int* stop, hipStream_t st,
                         double* da_out) {
  const int ch = row_chunks(s), stride = part_stride(s);
  k_update<<<dim3(s.N, ch), 256, 0, st>>>(s, A, b.P, b.G, b.Q, mu_host, state, Ac, b.rowpart, ch,
                                           stride, da_out, stop);
  return hipGetLastError();
}

hipError_t launch_update_reduce(const Shape& s, const SmallBuffers& b, double* scal_out,
                                const int* stop, hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride(s);
  k_rows_reduce<<<s.N + 1, 256, 0, st>>>(b.rowpart, s.N, ch, stride, s.R * s.R, b.Cc, scal_out, stop);
  return hipGetLastError();
}

hipError_t launch_als_rows(const Shape& s, int n, const double* M, const SmallBuffers& b, double* A,
                           hipStream_t st) {
  const long long total = (long long)s.I[n] * s.R;
  long long blocks = (total + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  k_als_rows<<<(unsigned)blocks, 256, 0, st>>>(s, n, M, b.Gt, A);
  return hipGetLastError();
}

}  // namespace dgn
