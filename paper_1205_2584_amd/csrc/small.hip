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
#include "panel.hpp"

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

// Products of small LDS matrices on the FP64 matrix cores.  Each 16 x 16
// result block (ti, tj), ti < mt, tj < nt, is formed by one wave (the waves
// take the blocks in turn) as out(i, j, sum_{k < K} a(i, k) b(k, j)), K a
// multiple of 4; the operands must be zero wherever i, j or k lies beyond the
// true sizes.  v_mfma_f64_16x16x4f64: lane l supplies a(16 ti + l%16, k + l/16)
// and b(k + l/16, 16 tj + l%16) and receives the result rows 16 ti + l/16 + 4v
// of column 16 tj + l%16.  Call from wave-uniform control flow.
template <typename FA, typename FB, typename FO>
__device__ __forceinline__ void mm16(int mt, int nt, int K, FA a, FB b, FO out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, cl = lane & 15, kq = lane >> 4;
  for (int tile = w; tile < mt * nt; tile += (int)(blockDim.x >> 6)) {
    const int ti = tile % mt, tj = tile / mt;
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = 0; k < K; k += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(16 * ti + cl, k + kq), b(k + kq, 16 * tj + cl), acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) out(16 * ti + kq + 4 * v, 16 * tj + cl, acc[v]);
  }
}

// R rounded up to a multiple of 16 (the MFMA block edge).
__device__ __forceinline__ int round16(int R) { return (R + 15) & ~15; }

// Zero S[i][j], i < 64, R <= j < Rp (the padding columns of a 64-row block).
__device__ __forceinline__ void pad_cols(double (*S)[LD], int R, int Rp) {
  for (int e = threadIdx.x; e < 64 * (Rp - R); e += blockDim.x) S[e & 63][R + (e >> 6)] = 0.0;
}

// Zero S[i][j], i, j < Rp, outside the leading R x R block.
__device__ __forceinline__ void pad_rr(double (*S)[LD], int R, int Rp) {
  for (int e = threadIdx.x; e < 64 * Rp; e += blockDim.x) {
    const int i = e & 63, j = e >> 6;
    if (i < Rp && (i >= R || j >= R)) S[i][j] = 0.0;
  }
}

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

// Rows r0..r0+63 of the column-major In x R block src, as the thread's share
// of S[ii][r] (zero outside): load_rows issues the loads, store_rows puts them
// into LDS (optionally adding the square-sum of the values to *sq), so that
// other loads can be issued in between.
struct RowVals {
  double v[16];
};
__device__ __forceinline__ void load_rows(RowVals& rv, const double* src, int In, int r0, int R) {
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, ii = e & 63, r = e >> 6;
    rv.v[s2] = (r < R && r0 + ii < In) ? src[r0 + ii + (long long)r * In] : 0.0;
  }
}
__device__ __forceinline__ void store_rows(double (*S)[LD], const RowVals& rv, int R, double* sq = nullptr) {
  double acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, ii = e & 63, r = e >> 6;
    if (r < R) S[ii][r] = rv.v[s2];
    acc += rv.v[s2] * rv.v[s2];
  }
  if (sq) *sq += acc;
}
__device__ __forceinline__ void stage_rows(double (*S)[LD], const double* src, int In, int r0, int R,
                                           double* sq = nullptr) {
  RowVals rv;
  load_rows(rv, src, In, r0, R);
  store_rows(S, rv, R, sq);
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

// Factor an Rp x Rp block (Rp = 16 nkb) held in T rows 0..Rp-1 in place by the
// first wave: per 16-column step the L D L^T of the diagonal block, the
// triangular solve of the rows below it and the MFMA update of the blocks to
// its right.  PSD: semidefinite-safe, with the original diagonal in dref.
template <bool PSD>
__device__ void chol_chain(double (*T)[TR], int nkb, int* bad, double (*Lk)[16][16], double* rinv,
                           const double* dref) {
  const int lane = threadIdx.x & 63, Rp = 16 * nkb;
  for (int kb = 0; kb < nkb; ++kb) {
    const int k0 = 16 * kb;
    chol16<PSD>(T, k0, bad, Lk[kb], rinv, dref);
    if (lane < Rp - k0 - 16) trsm16_row(T, k0 + 16 + lane, k0, Lk[kb], rinv);
    for (int bi = kb + 1; bi < nkb; ++bi)
      for (int bj = kb + 1; bj <= bi; ++bj) trail16(T, bi, bj, k0);
  }
}

// Per mode n (blockIdx.y = 0): Gamma_n, the Cholesky factor L of Gamma_n + mu I,
// X_n = L^-T and Gt_n = X_n X_n^T = (Gamma_n + mu I)^-1; a non-positive pivot
// sets *bad.  blockIdx.y = 1: the semidefinite-safe Cholesky factor L_n of C_n
// (a pivot below 64 u times its original diagonal drops its column).  The R x R
// matrix is the leading block of a 64 x 64 LDS tile completed with the
// identity; the first wave factors it and the workgroup inverts the factor.
__global__ __launch_bounds__(256) void k_gamma(Shape s, const double* C, double mu_host,
                                               const FitState* state, double* Gam, double* Gt,
                                               double* X, double* Lc, int* bad, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double T[128][TR];                   // rows 0..63: H, then L; rows 64..127: L^-1
  __shared__ __align__(16) double Lk[4][16][16];  // L_kk of each column step, then scratch
  __shared__ double rinv[64];                     // 1 / L_kk
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  const int nkb = (R + 15) >> 4, Rp = 16 * nkb;
  const bool chol_c = blockIdx.y == 1;
  RR_SHIFT;
  const double mu = state ? state->mu : mu_host;
  double* dref = &T[64][0];  // original diagonal of C_n (the semidefinite factor only)
  if (chol_c) {
    for_rr_staged(
        R, rr_sh, [&](int r, int q) { return C[(long long)n * R2 + r + q * R]; },
        [&](int r, int q, double v) { T[r][q] = v; });
    for (int r = t; r < 64; r += 256) dref[r] = r < R ? C[(long long)n * R2 + r + r * R] : 1.0;
  } else {
    for_rr_staged(
        R, rr_sh,
        [&](int r, int q) {
          double cv[kMaxOrder];
          load_c(C, N, R2, r + q * R, cv);
          return prod_except(cv, n, -1);
        },
        [&](int r, int q, double g) {
          Gam[(long long)n * R2 + r + q * R] = g;
          T[r][q] = g + (r == q ? mu : 0.0);
        });
  }
  for (int e = t; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    if (r >= R || c >= R) T[r][c] = (r == c) ? 1.0 : 0.0;
    if (!chol_c) T[64 + r][c] = 0.0;  // the inverse writes its lower blocks only
  }
  sync_block();
  if (t < 64) {
    if (chol_c)
      chol_chain<true>(T, nkb, bad, Lk, rinv, dref);
    else
      chol_chain<false>(T, nkb, bad, Lk, rinv, nullptr);
    if (t >= Rp) rinv[t] = 1.0;
  }
  sync_block();
  if (chol_c) {
    // the blocks above the diagonal still hold C
    FOR_RR(r, q) Lc[(long long)n * R2 + r + q * R] = (r >= q) ? T[r][q] : 0.0;
    return;
  }
  invert_lower64(T, T + 64, rinv, Lk, nkb);
  // X = L^-T (upper triangular), Gt = L^-T L^-1 (the padding rows of L^-1 are
  // zero in the first R columns, so the sum may run to Rp)
  FOR_RR(r, q) X[(long long)n * R2 + r + q * R] = T[64 + q][r];
  mm16(
      nkb, nkb, Rp, [&](int r, int k) { return T[64 + k][r]; }, [&](int k, int q) { return T[64 + k][q]; },
      [&](int r, int q, double v) {
        if (r < R && q < R) Gt[(long long)n * R2 + r + q * R] = v;
      });
}

// Rows of mode n, chunk c: G = M - A Gamma (or M itself when it already is the
// gradient), P = G Gt, partial w = A^T P, partial ||G||^2 and ||M||^2.  The
// three products run on the matrix cores with R padded to Rp = 16 ceil(R/16).
__device__ void pw_block(const Shape& s, int n, int c, const double* A, const double* M, int resid,
                         const double* Gam, const double* Gt, double* Gout, double* Pout, double* part,
                         int chunks, int stride, double (*As)[LD], double (*Gs)[LD], double (*Ps)[LD],
                         double (*Gm)[LD], double* red) {
  const int R = s.R, R2 = R * R, In = s.I[n], t = threadIdx.x, nt = (R + 15) >> 4, Rp = 16 * nt;
  RR_SHIFT;
  const int r0 = c * 64;
  double* out = part + ((long long)n * chunks + c) * stride;
  if (r0 >= In) {
    for (int e = t; e < R2 + 4; e += 256) out[e] = 0.0;
    return;
  }
  const long long base = (long long)s.off[n] * R;
  const double* G0 = (resid ? Gt : Gam) + (long long)n * R2;
  // the row loads of A and M in flight while Gamma (or Gt) is staged
  RowVals ra, rm;
  load_rows(ra, A + base, In, r0, R);
  load_rows(rm, M + base, In, r0, R);
  for_rr_staged(
      R, rr_sh, [&](int r, int q) { return G0[r + q * R]; }, [&](int r, int q, double v) { Gm[r][q] = v; });
  double m2 = 0.0;
  store_rows(As, ra, R);
  store_rows(Gs, rm, R, &m2);
  pad_cols(As, R, Rp);
  pad_cols(Gs, R, Rp);
  pad_rr(Gm, R, Rp);
  sync_block();
  double (*Gp)[LD] = Gs;  // gradient rows
  double (*Pp)[LD] = Ps;  // rows of P
  if (!resid) {
    // G = M - A Gamma, into Ps
    mm16(
        4, nt, Rp, [&](int i, int k) { return As[i][k]; }, [&](int k, int j) { return Gm[k][j]; },
        [&](int i, int j, double v) { Ps[i][j] = Gs[i][j] - v; });
    sync_block();
    for_rr_staged(
        R, rr_sh, [&](int r, int q) { return Gt[(long long)n * R2 + r + q * R]; },
        [&](int r, int q, double v) { Gm[r][q] = v; });
    sync_block();
    Gp = Ps;
    Pp = Gs;
  }
  mm16(
      4, nt, Rp, [&](int i, int k) { return Gp[i][k]; }, [&](int k, int j) { return Gm[k][j]; },
      [&](int i, int j, double v) { Pp[i][j] = v; });
  sync_block();
  double g2 = 0.0;
  for (int e = t; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    if (r0 + ii < In) {
      const long long gi = base + r0 + ii + (long long)r * In;
      const double g = Gp[ii][r];
      Gout[gi] = g;
      Pout[gi] = Pp[ii][r];
      g2 += g * g;
    }
  }
  // partial w = A^T P over the chunk's rows (rows beyond I_n are zero in both)
  mm16(
      nt, nt, 64, [&](int a, int k) { return As[k][a]; }, [&](int k, int b) { return Pp[k][b]; },
      [&](int a, int b, double v) {
        if (a < R && b < R) out[a + b * R] = v;
      });
  g2 = block_sum(g2, red);
  m2 = block_sum(m2, red);
  if (t == 0) {
    out[R2 + 0] = g2;
    out[R2 + 1] = m2;
    out[R2 + 2] = 0.0;
    out[R2 + 3] = 0.0;
  }
}

// T_nm[(a + d R) * R + i] = sum_j Gamma_nm[i, j] L_n[j, a] X_m[j, d] for n != m
// and one d.
__device__ void tnm_block(const Shape& s, int pair, int d, const double* C, const double* X,
                          const double* Lc, double* Tnm, double (*Gs)[LD], double (*Ls)[LD]) {
  const int R = s.R, R2 = R * R, N = s.N, nt = (R + 15) >> 4, Rp = 16 * nt;
  RR_SHIFT;
  const int n = pair / N, m = pair % N;
  const double* xd = X + (long long)m * R2 + d * R;  // X_m[:, d]
  // Ls[j][a] = L_n[j, a] X_m[j, d]
  for_rr_staged(
      R, rr_sh,
      [&](int i, int j) {
        const int e = i + j * R;
        double cv[kMaxOrder];
        load_c(C, N, R2, e, cv);
        return d3{prod_except(cv, n, m), Lc[(long long)n * R2 + e], xd[i]};
      },
      [&](int i, int j, d3 v) {
        Gs[i][j] = v.x;
        Ls[i][j] = v.y * v.z;
      });
  pad_rr(Gs, R, Rp);
  pad_rr(Ls, R, Rp);
  sync_block();
  double* out = Tnm + (long long)pair * R * R2;
  mm16(
      nt, nt, Rp, [&](int i, int j) { return Gs[i][j]; }, [&](int j, int a) { return Ls[j][a]; },
      [&](int i, int a, double v) {
        if (i < R && a < R) out[((long long)a + (long long)d * R) * R + i] = v;
      });
}

// Blocks 0 .. N chunks - 1: the rows of the fast step's gradient (pw_block).
// With tnm, the N (N - 1) R blocks after them form the T_nm of the NR^2
// assembly (they need only C, X and L from k_gamma).
__global__ __launch_bounds__(256) void k_pw(Shape s, const double* A, const double* M, int resid,
                                            const double* Gam, const double* Gt, double* Gout,
                                            double* Pout, double* part, int chunks, int stride,
                                            const double* C, const double* X, const double* Lc,
                                            double* Tnm, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double As[64][LD];
  __shared__ double Gs[64][LD];
  __shared__ double Ps[64][LD];
  __shared__ double Gm[64][LD];
  __shared__ double red[16];
  const int id = blockIdx.x, npw = s.N * chunks;
  if (id < npw) {
    pw_block(s, id / chunks, id % chunks, A, M, resid, Gam, Gt, Gout, Pout, part, chunks, stride, As, Gs, Ps,
             Gm, red);
    return;
  }
  // T_nm blocks: pairs n != m in order, then d
  const int R = s.R, k = id - npw, p = k / R, d = k % R;
  const int n = p / (s.N - 1), mo = p % (s.N - 1), m = mo < n ? mo : mo + 1;
  tnm_block(s, n * s.N + m, d, C, X, Lc, Tnm, As, Gs);
}

// w_m[e] = sum over the row chunks of the partials A_m^T P_m, eight loads in
// flight at a time.
__device__ __forceinline__ double w_sum(const double* part, int m, int chunks, int stride, int e) {
  const double* p0 = part + (long long)m * chunks * stride + e;
  double acc = 0.0;
  int c = 0;
  for (; c + 8 <= chunks; c += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p0[(long long)(c + k) * stride];
    acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
  for (; c < chunks; ++c) acc += p0[(long long)c * stride];
  return acc;
}

// w = the sums of the row-chunk partials A_n^T P_n, one entry per thread over
// all modes; the last block reduces ||G||^2 and ||M||^2 into scal[2], scal[3].
__global__ __launch_bounds__(256) void k_wred(Shape s, const double* part, int chunks, int stride, double* w,
                                              double* scal, const int* stop) {
  if (stopped(stop)) return;
  const int R2 = s.R * s.R, N = s.N, t = threadIdx.x;
  if ((int)blockIdx.x == (int)gridDim.x - 1) {
    if (t < 2) {
      double acc = 0.0;
      for (int m = 0; m < N; ++m)
        for (int c = 0; c < chunks; ++c) acc += part[((long long)m * chunks + c) * stride + R2 + t];
      scal[2 + t] = acc;
    }
    return;
  }
  const int x = blockIdx.x * 256 + t;
  if (x < N * R2) w[x] = w_sum(part, x / R2, chunks, stride, x % R2);
}

// Per mode n: V = sum_{m != n} Gamma_nm * W_m^T and z_n = vec(L_n^T V X_n)
// (= (W^T K w)_n).
__global__ __launch_bounds__(256) void k_z(Shape s, const double* C, const double* w, const double* X,
                                           const double* Lc, double* z, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double V[64][LD];
  __shared__ double Ls[64][LD];
  __shared__ double Xs[64][LD];
  __shared__ double Tm[64][LD];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, nt = (R + 15) >> 4, Rp = 16 * nt;
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
  pad_rr(V, R, Rp);
  pad_rr(Ls, R, Rp);
  pad_rr(Xs, R, Rp);
  sync_block();
  // Tm = L_n^T V
  mm16(
      nt, nt, Rp, [&](int a, int k) { return Ls[k][a]; }, [&](int k, int b) { return V[k][b]; },
      [&](int a, int b, double v) { Tm[a][b] = v; });
  sync_block();
  mm16(
      nt, nt, Rp, [&](int a, int k) { return Tm[a][k]; }, [&](int k, int b) { return Xs[k][b]; },
      [&](int a, int b, double v) {
        if (a < R && b < R) z[(long long)n * R2 + a + b * R] = v;
      });
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
  const int n = blockIdx.x, R = s.R, R2 = R * R, nt = (R + 15) >> 4, Rp = 16 * nt;
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
  pad_rr(Ys, R, Rp);
  pad_rr(Ls, R, Rp);
  pad_rr(Xs, R, Rp);
  sync_block();
  mm16(
      nt, nt, Rp, [&](int a, int k) { return Ls[a][k]; }, [&](int k, int b) { return Ys[k][b]; },
      [&](int a, int b, double v) { Tm[a][b] = v; });
  sync_block();
  mm16(
      nt, nt, Rp, [&](int a, int k) { return Tm[a][k]; }, [&](int k, int b) { return Xs[b][k]; },
      [&](int a, int b, double v) {
        if (a < R && b < R) {
          const long long e = (long long)n * R2 + a + b * R;
          u[e] = w[e] - v;
        }
      });
}

// f_n = vec(sum_{m != n} Gamma_nm * U_m^T) (= (K u)_n), Q_n = F_n Gt_n.
__global__ __launch_bounds__(256) void k_fq(Shape s, const double* C, const double* u,
                                            const double* Gt, double* f, double* Q,
                                            const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Fs[64][LD];
  __shared__ double Gs[64][LD];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, nt = (R + 15) >> 4, Rp = 16 * nt;
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
  pad_rr(Fs, R, Rp);
  pad_rr(Gs, R, Rp);
  sync_block();
  mm16(
      nt, nt, Rp, [&](int a, int k) { return Fs[a][k]; }, [&](int k, int b) { return Gs[k][b]; },
      [&](int a, int b, double v) {
        if (a < R && b < R) Q[(long long)n * R2 + a + b * R] = v;
      });
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
  const int nt = (R + 15) >> 4, Rp = 16 * nt;
  RR_SHIFT;
  const int r0 = c * 64;
  double* out = part + ((long long)n * chunks + c) * stride;
  if (r0 >= In) {
    for (int e = t; e < R2 + 4; e += 256) out[e] = 0.0;
    return;
  }
  const double mu = state ? state->mu : mu_host;
  const long long base = (long long)s.off[n] * R;
  // this thread's entries of P and G, in flight while A and Q_n are staged
  constexpr int NE = 64 * kMaxRank / 256;
  double pv[NE], gv[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = t + 256 * k, ii = e & 63, r = e >> 6;
    const bool ok = e < 64 * R && r0 + ii < In;
    const long long gi = base + r0 + ii + (long long)r * In;
    pv[k] = ok ? P[gi] : 0.0;
    gv[k] = ok ? G[gi] : 0.0;
  }
  RowVals ra;
  load_rows(ra, A + base, In, r0, R);
  for_rr_staged(
      R, rr_sh, [&](int r, int q) { return Q[(long long)n * R2 + r + q * R]; },
      [&](int r, int q, double v) { Qs[r][q] = v; });
  store_rows(As, ra, R);
  pad_cols(As, R, Rp);
  pad_rr(Qs, R, Rp);
  sync_block();
  // Cs = A Q_n (padding columns come out zero)
  mm16(
      4, nt, Rp, [&](int i, int k) { return As[i][k]; }, [&](int k, int j) { return Qs[k][j]; },
      [&](int i, int j, double v) { Cs[i][j] = v; });
  sync_block();
  double den = 0.0, da2 = 0.0;
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = t + 256 * k, ii = e & 63, r = e >> 6;
    if (e < 64 * R) {
      double v = 0.0;
      if (r0 + ii < In) {
        const long long gi = base + r0 + ii + (long long)r * In;
        const double da = pv[k] - Cs[ii][r];
        v = As[ii][r] + da;
        Ac[gi] = v;
        if (da_out) da_out[gi] = da;
        den += da * (gv[k] + mu * da);
        da2 += da * da;
      }
      Cs[ii][r] = v;
    }
  }
  sync_block();
  mm16(
      nt, nt, 64, [&](int a, int k) { return Cs[k][a]; }, [&](int k, int b) { return Cs[k][b]; },
      [&](int a, int b, double v) {
        if (a < R && b < R) out[a + b * R] = v;
      });
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
                     const SmallBuffers& b, bool with_tnm, const int* stop, hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride(s);
  const int nblk = s.N * ch + (with_tnm ? s.N * (s.N - 1) * s.R : 0);
  k_pw<<<nblk, 256, 0, st>>>(s, A, M, resid ? 1 : 0, b.Gam, b.Gt, b.G, b.P, b.wpart, ch, stride, b.C, b.X, b.Lc,
                             b.Tnm, stop);
  return hipGetLastError();
}

hipError_t launch_wz(const Shape& s, const SmallBuffers& b, const int* stop, hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride(s);
  const int nw = (s.N * s.R * s.R + 255) / 256;
  k_wred<<<nw + 1, 256, 0, st>>>(s, b.wpart, ch, stride, b.w, b.scal, stop);
  k_z<<<s.N, 256, 0, st>>>(s, b.C, b.w, b.X, b.Lc, b.z, stop);
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
