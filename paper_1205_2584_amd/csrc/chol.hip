// The NR^2 system of the fast step in symmetric positive definite form.
//
// With W = blkdiag(X_n (x) L_n) (X_n X_n^T = Gt_n, L_n L_n^T = C_n) the fLMa
// system (I + Psi K) x = w of Section 4.3 is similar to S = I + W^T K W,
// which is SPD because H + mu I is (the eigenvalues of S are those of
// I + Psi K, i.e. of the damped Hessian's Woodbury capacitance).  Blocks,
// with p = n R^2 + a + b R:
//   S_nn = I,   S_nm[a + bR, c + dR] = sum_i X_n[i,b] L_m[i,c] T_nm[i, a + dR],
//   T_nm[i, a + dR] = sum_j Gamma_nm[i,j] L_n[j,a] X_m[j,d].
// The identity block of mode 1 is eliminated first (its factor column is the
// block column B itself), leaving the trailing system
//   (S_tt - B B^T) y_t = z_t - B z_1,   y_1 = z_1 - B^T y_t,
// which is factored by a tiled right-looking Cholesky (64 x 64 FP64 tiles,
// MFMA trailing updates).  The right-hand side rides along as an extra tile
// row, so the forward substitution happens inside the factorisation; the
// backward substitution runs tile by tile afterwards.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int LD = kMaxRank + 1;
constexpr int TL = 65;  // padded leading dimension of 64 x 64 LDS tiles

// acc[blk] (wave w owns rows 16w..16w+15 of a 64 x 64 tile; blk selects 16
// columns) += A(rows) * B(cols)^T over k < K (K a multiple of 4).
// A and B are column-major with leading dimensions lda / ldb.
// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16] and the
// result D[l/16 + 4v][l%16], v = 0..3.
__device__ __forceinline__ void mma_tile(const double* __restrict__ A, long long lda,
                                         const double* __restrict__ B, long long ldb, int K,
                                         v4d acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* ap = A + 16 * w + (lane & 15) + (long long)(lane >> 4) * lda;
  const double* bp = B + (lane & 15) + (long long)(lane >> 4) * ldb;
  for (int k = 0; k < K; k += 4) {
    const double a = ap[(long long)k * lda];
    double b[4];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) b[blk] = bp[16 * blk + (long long)k * ldb];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) acc[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[blk], acc[blk], 0, 0, 0);
  }
}

__device__ __forceinline__ int acc_row(int v) { return 16 * (threadIdx.x >> 6) + ((threadIdx.x & 63) >> 4) + 4 * v; }
__device__ __forceinline__ int acc_col(int blk) { return 16 * blk + (threadIdx.x & 15); }

__device__ __forceinline__ void zero_acc(v4d acc[4]) {
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
}

// 64 x 64 Cholesky of the lower triangle of D (LDS) in place; bad pivots flag *bad.
__device__ void chol64(double (*D)[TL], double* lk, int* bad) {
  const int t = threadIdx.x;
  for (int k = 0; k < 64; ++k) {
    __syncthreads();
    const double dkk = D[k][k];
    double d = 1.0;
    if (dkk > 0.0) d = sqrt(dkk);
    else if (t == 0) *bad = 1;
    if (t >= k && t < 64) lk[t] = (t == k) ? d : D[t][k] / d;
    __syncthreads();
    const int m = 63 - k;
    for (int e = t; e < m * m; e += 256) {
      const int i = k + 1 + e % m, j = k + 1 + e / m;
      if (j <= i) D[i][j] -= lk[i] * lk[j];
    }
    if (t >= k && t < 64) D[t][k] = lk[t];
  }
  __syncthreads();
}

// X = Bt * L^-T for the 64 x 64 tile Bt (LDS, overwritten with X); L lower (LDS).
// Four lanes share a row; each holds the columns congruent to its lane mod 4.
__device__ void trsm64(double (*Bt)[TL], double (*L)[TL]) {
  const int t = threadIdx.x, row = t >> 2, sub = t & 3;
  double x[16];
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (4 * q + sub < c) part += x[q] * L[c][4 * q + sub];
    part += __shfl_xor(part, 1, 64);
    part += __shfl_xor(part, 2, 64);
    const double v = (Bt[row][c] - part) / L[c][c];
    if ((c & 3) == sub) x[c >> 2] = v;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) Bt[row][4 * q + sub] = x[q];
  __syncthreads();
}

// Fill the lower tiles of St and all of B with identity / zeros (the
// off-diagonal blocks are overwritten by k_subblock afterwards).
__global__ __launch_bounds__(256) void k_fill(SysPlan p, double* St, double* B, int R2p,
                                              const int* stop) {
  if (stopped(stop)) return;
  const long long ntri = (long long)p.Tt * (p.Tt + 1) / 2 + p.Tt;  // lower tiles + RHS row tiles
  const long long id = blockIdx.x;
  if (id < ntri) {
    int ti, tj;
    if (id < (long long)p.Tt * (p.Tt + 1) / 2) {
      ti = (int)((sqrt(8.0 * id + 1.0) - 1.0) / 2.0);
      while ((long long)(ti + 1) * (ti + 2) / 2 <= id) ++ti;
      while ((long long)ti * (ti + 1) / 2 > id) --ti;
      tj = (int)(id - (long long)ti * (ti + 1) / 2);
    } else {
      ti = p.Tt;
      tj = (int)(id - (long long)p.Tt * (p.Tt + 1) / 2);
    }
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int ii = e & 63, jj = e >> 6;
      const int r = ti * 64 + ii, c = tj * 64 + jj;
      double v = 0.0;
      if (ti < p.Tt && r == c) v = 1.0;
      St[r + (long long)c * p.lds] = v;
    }
  } else {
    const long long nb = (long long)p.ntp * R2p;
    for (long long e = (id - ntri) * 256 + threadIdx.x; e < nb; e += (long long)(gridDim.x - ntri) * 256)
      B[e] = 0.0;
  }
}

// R x R sub-block (b, d) of S_nm for n > m: rows n R^2 + a + b R, columns m R^2 + c + d R.
__global__ __launch_bounds__(256) void k_subblock(Shape s, SysPlan p, const double* Tnm,
                                                  const double* X, const double* Lc, double* St,
                                                  double* B, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Td[64][LD];  // Td[i][a] = T_nm[i, a + dR]
  __shared__ double Lm[64][LD];
  __shared__ double xb[64];
  const int N = s.N, R = s.R, R2 = R * R;
  // decode the strictly lower pair (n, m), n > m
  int pr = blockIdx.x / R, b = blockIdx.x % R, d = blockIdx.y;
  int n = 1, m = 0;
  while (pr >= n) { pr -= n; ++n; }
  m = pr;
  (void)N;
  const int pair = n * N + m;
  const double* T = Tnm + (long long)pair * R * R2;
  for (int e = threadIdx.x; e < R2; e += 256) {
    const int i = e % R, a = e / R;
    Td[i][a] = T[((long long)a + (long long)d * R) * R + i];
    Lm[i][a] = Lc[(long long)m * R2 + e];  // Lm[i][c] = L_m[i, c]
  }
  for (int i = threadIdx.x; i < R; i += 256) xb[i] = X[(long long)n * R2 + i + b * R];
  __syncthreads();
  for (int e = threadIdx.x; e < R2; e += 256) {
    const int a = e % R, c = e / R;
    double acc = 0.0;
    for (int i = 0; i < R; ++i) acc += Td[i][a] * xb[i] * Lm[i][c];
    const long long row = (long long)(n - 1) * R2 + a + b * R;  // trailing row index
    if (m == 0) {
      B[row + (long long)(c + d * R) * p.ntp] = acc;
    } else {
      const long long col = (long long)(m - 1) * R2 + c + d * R;
      St[row + col * p.lds] = acc;
    }
  }
}

// Right-hand side row: St[ntp, q] = z_t[q] - (B z_1)[q].
__global__ void k_rhs(SysPlan p, const double* B, const double* z, double* St, const int* stop) {
  if (stopped(stop)) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= p.ntp) return;
  double v = 0.0;
  if (q < p.nt) {
    v = z[p.R2 + q];
    for (int k = 0; k < p.R2; ++k) v -= B[q + (long long)k * p.ntp] * z[k];
  }
  St[p.ntp + (long long)q * p.lds] = v;
}

__device__ __forceinline__ void tri_index(long long id, int& ti, int& tj) {
  ti = (int)((sqrt(8.0 * id + 1.0) - 1.0) / 2.0);
  while ((long long)(ti + 1) * (ti + 2) / 2 <= id) ++ti;
  while ((long long)ti * (ti + 1) / 2 > id) --ti;
  tj = (int)(id - (long long)ti * (ti + 1) / 2);
}

// St_tt -= B B^T on the lower tiles (K = R2p, a multiple of 4).
__global__ __launch_bounds__(256) void k_syrk(SysPlan p, const double* B, int R2p, double* St,
                                              const int* stop) {
  if (stopped(stop)) return;
  int ti, tj;
  tri_index(blockIdx.x, ti, tj);
  v4d acc[4];
  zero_acc(acc);
  mma_tile(B + ti * 64, p.ntp, B + tj * 64, p.ntp, R2p, acc);
  double* C = St + ti * 64 + (long long)tj * 64 * p.lds;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk)
#pragma unroll
    for (int v = 0; v < 4; ++v) C[acc_row(v) + (long long)acc_col(blk) * p.lds] -= acc[blk][v];
}

// Phase ph of the tiled Cholesky.  Blocks [0, Tt - ph + 1): panel row tiles
// i = ph + blk (the last one being the right-hand-side row); each applies the
// update of column ph-1 to its tile and to the diagonal tile, factors the
// diagonal tile and solves its tile.  Remaining blocks: trailing tiles
// (i, j), ph < j <= i <= Tt, j < Tt, receive the update of column ph-1.
__global__ __launch_bounds__(256) void k_chol_phase(SysPlan p, int ph, double* St, int* bad,
                                                    const int* stop) {
  if (stopped(stop)) return;
  __shared__ double D[64][TL];
  __shared__ double Bt[64][TL];
  __shared__ double lk[64];
  const int npanel = p.Tt - ph + 1;
  const long long lds = p.lds;
  const int t = threadIdx.x;
  if ((int)blockIdx.x < npanel) {
    const int i = ph + blockIdx.x;
    double* Dg = St + ph * 64 + (long long)ph * 64 * lds;
    double* Bg = St + i * 64 + (long long)ph * 64 * lds;
    for (int e = t; e < 64 * 64; e += 256) {
      const int r = e & 63, c = e >> 6;
      D[r][c] = Dg[r + c * lds];
      if (i != ph) Bt[r][c] = Bg[r + c * lds];
    }
    __syncthreads();
    if (ph > 0) {
      const double* Lp = St + ph * 64 + (long long)(ph - 1) * 64 * lds;   // L(ph, ph-1)
      v4d acc[4];
      zero_acc(acc);
      mma_tile(Lp, lds, Lp, lds, 64, acc);
#pragma unroll
      for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int v = 0; v < 4; ++v) D[acc_row(v)][acc_col(blk)] -= acc[blk][v];
      if (i != ph) {
        const double* Li = St + i * 64 + (long long)(ph - 1) * 64 * lds;  // L(i, ph-1)
        zero_acc(acc);
        mma_tile(Li, lds, Lp, lds, 64, acc);
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
#pragma unroll
          for (int v = 0; v < 4; ++v) Bt[acc_row(v)][acc_col(blk)] -= acc[blk][v];
      }
    }
    chol64(D, lk, bad);
    if (i == ph) {
      for (int e = t; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        Dg[r + c * lds] = (c <= r) ? D[r][c] : 0.0;
      }
    } else {
      trsm64(Bt, D);
      for (int e = t; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        Bg[r + c * lds] = Bt[r][c];
      }
    }
    return;
  }
  // trailing update with column ph - 1
  if (ph == 0) return;
  long long id = (long long)blockIdx.x - npanel;
  // enumerate (i, j): j from ph+1 to Tt-1, i from j to Tt
  int j = ph + 1;
  while (id >= (long long)(p.Tt - j + 1)) { id -= (p.Tt - j + 1); ++j; }
  const int i = j + (int)id;
  const double* Li = St + i * 64 + (long long)(ph - 1) * 64 * lds;
  const double* Lj = St + j * 64 + (long long)(ph - 1) * 64 * lds;
  v4d acc[4];
  zero_acc(acc);
  mma_tile(Li, lds, Lj, lds, 64, acc);
  double* C = St + i * 64 + (long long)j * 64 * lds;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk)
#pragma unroll
    for (int v = 0; v < 4; ++v) C[acc_row(v) + (long long)acc_col(blk) * lds] -= acc[blk][v];
}

// Backward substitution, phase k (descending): every block solves
// L_kk^T y_k = u_k (u in the RHS row); block k stores y_k, block j < k
// updates u_j -= L_kj^T y_k.
__global__ __launch_bounds__(256) void k_bsolve(SysPlan p, int k, double* St, double* yt,
                                                const int* stop) {
  if (stopped(stop)) return;
  __shared__ double L[64][TL];
  __shared__ double ys[64];
  const long long lds = p.lds;
  const int t = threadIdx.x, j = blockIdx.x;
  const double* Lg = St + k * 64 + (long long)k * 64 * lds;
  for (int e = t; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    L[r][c] = Lg[r + c * lds];
  }
  __syncthreads();
  if (t < 64) {
    // lane c holds u_k[c]; sweep c = 63..0
    double val = St[p.ntp + (long long)(k * 64 + t) * lds];
    double y = 0.0;
    for (int c = 63; c >= 0; --c) {
      const double yc = __shfl(val / L[c][c], c, 64);
      if (t == c) y = yc;
      if (t < c) val -= L[c][t] * yc;
    }
    ys[t] = y;
  }
  __syncthreads();
  if (j == k) {
    if (t < 64) yt[k * 64 + t] = ys[t];
    return;
  }
  // u_j[c] -= sum_r L(k, j)[r][c] y_k[r]
  const double* Lkj = St + k * 64 + (long long)j * 64 * lds;
  if (t < 64) {
    double acc = 0.0;
    for (int r = 0; r < 64; ++r) acc += Lkj[r + (long long)t * lds] * ys[r];
    St[p.ntp + (long long)(j * 64 + t) * lds] -= acc;
  }
}

// y_1 = z_1 - B^T y_t (one wave per entry) and y[R^2 + q] = y_t[q].
__global__ __launch_bounds__(256) void k_y0(SysPlan p, const double* B, const double* z,
                                            const double* yt, double* y, const int* stop) {
  if (stopped(stop)) return;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k < p.R2) {
    double acc = 0.0;
    for (int q = lane; q < p.nt; q += 64) acc += B[q + (long long)k * p.ntp] * yt[q];
    acc = wave_sum(acc);
    if (lane == 0) y[k] = z[k] - acc;
  }
  for (int q = blockIdx.x * 256 + threadIdx.x; q < p.nt; q += gridDim.x * 256) y[p.R2 + q] = yt[q];
}

}  // namespace

SysPlan plan_sys(const Shape& s) {
  SysPlan p{};
  p.R2 = s.R * s.R;
  p.nt = (s.N - 1) * p.R2;
  p.ntp = ((p.nt + 63) / 64) * 64;
  p.Tt = p.ntp / 64;
  p.lds = p.ntp + 64;
  return p;
}

static inline int r2pad(int R2) { return ((R2 + 3) / 4) * 4; }

hipError_t launch_sys_assemble(const Shape& s, const SysPlan& p, const SmallBuffers& b,
                               const SysBuffers& y, const int* stop, hipStream_t st) {
  const int R2p = r2pad(p.R2);
  const long long ntri = (long long)p.Tt * (p.Tt + 1) / 2 + p.Tt;
  const long long nbblocks = ((long long)p.ntp * R2p + 255) / 256;
  long long extra = nbblocks < 1024 ? nbblocks : 1024;
  k_fill<<<(unsigned)(ntri + extra), 256, 0, st>>>(p, y.St, y.B, R2p, stop);
  const int npairs = s.N * (s.N - 1) / 2;
  k_subblock<<<dim3(npairs * s.R, s.R), 256, 0, st>>>(s, p, b.Tnm, b.X, b.Lc, y.St, y.B, stop);
  k_rhs<<<(p.ntp + 255) / 256, 256, 0, st>>>(p, y.B, b.z, y.St, stop);
  k_syrk<<<(unsigned)((long long)p.Tt * (p.Tt + 1) / 2), 256, 0, st>>>(p, y.B, R2p, y.St, stop);
  return hipGetLastError();
}

hipError_t launch_sys_factor_solve(const Shape& s, const SysPlan& p, const SmallBuffers& b,
                                   const SysBuffers& y, int* singular, const int* stop,
                                   hipStream_t st) {
  (void)s;
  for (int ph = 0; ph < p.Tt; ++ph) {
    const int npanel = p.Tt - ph + 1;
    long long nupd = 0;
    if (ph > 0)
      for (int j = ph + 1; j < p.Tt; ++j) nupd += p.Tt - j + 1;
    k_chol_phase<<<(unsigned)(npanel + nupd), 256, 0, st>>>(p, ph, y.St, singular, stop);
  }
  for (int k = p.Tt - 1; k >= 0; --k) k_bsolve<<<k + 1, 256, 0, st>>>(p, k, y.St, y.yt, stop);
  k_y0<<<(p.R2 + 3) / 4, 256, 0, st>>>(p, y.B, b.z, y.yt, b.y, stop);
  return hipGetLastError();
}

}  // namespace dgn
