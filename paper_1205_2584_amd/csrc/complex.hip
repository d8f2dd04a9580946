// The complex fast step (Section 5) on FP64 complex factors.
//
// Complex CP model: Y_hat = sum_r a_r^(1) o ... o a_r^(N) with complex factors,
// C_n = A_n^H A_n (Hermitian), Gamma_n and Gamma_nm Hadamard products of the
// C_k as in the real case.  With Gt_n = (Gamma_n + mu I)^-1:
//   M_n = Y_(n) (Khatri-Rao of conj(A_k), k != n)      (Theorem 5.4)
//   G_n = M_n - A_n Gamma_n^T,  P_n = G_n conj(Gt_n)    (the factor-side
//         inverse (Gamma_n^T + mu I)^-1 = Gt_n^T = conj(Gt_n), Gt_n Hermitian)
//   w_n = vec(A_n^H P_n),  Psi_n = Gt_n (x) C_n,  K_nm = P_R diag(vec Gamma_nm)
//   f = K (I + Psi K)^-1 w,  A_n <- A_n + P_n - A_n F_n conj(Gt_n).
// As in the real case the system is solved in the Hermitian positive definite
// form S = I + W^H K W, W = blkdiag(X_n (x) L_n), X_n X_n^H = Gt_n,
// L_n L_n^H = C_n, with the closed forms
//   S_nm[a + bR, c + dR] = sum_j conj(X_n[j,b]) L_m[j,c] T_nm[j, a + dR],
//   T_nm[j, a + dR]      = sum_i Gamma_nm[j,i] conj(L_n[i,a]) X_m[i,d],
//   z_n = vec(L_n^H (sum_m Gamma_nm^T * W_m^T) conj(X_n)),
//   u_n = w_n - vec(L_n Y_n X_n^T),  F_n = sum_m Gamma_nm^T * U_m^T.
// The trailing system (modes 2..N after eliminating the identity block of
// mode 1) is handed to the real tiled Cholesky through its real embedding
// [[Re S, -Im S], [Im S, Re S]], which is symmetric positive definite: the
// sub-block kernel writes the embedded entries, z and y use the embedded
// layout [Re z_1, Im z_1, Re z_t, Im z_t], and the block column B is stored as
// [[Re B, -Im B], [Im B, Re B]].
//
// Complex arrays are interleaved (re, im) FP64 pairs in the stacked layouts of
// the real path; the rank is limited to kMaxRankC.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

struct cd {
  double x, y;
};
__device__ __forceinline__ cd operator+(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd operator*(double s, cd a) { return cd{s * a.x, s * a.y}; }
__device__ __forceinline__ cd& operator+=(cd& a, cd b) {
  a.x += b.x;
  a.y += b.y;
  return a;
}
__device__ __forceinline__ cd& operator-=(cd& a, cd b) {
  a.x -= b.x;
  a.y -= b.y;
  return a;
}
__device__ __forceinline__ cd conjc(cd a) { return cd{a.x, -a.y}; }
__device__ __forceinline__ double abs2(cd a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ cd czero() { return cd{0.0, 0.0}; }
__device__ __forceinline__ cd shfl_xor_cd(cd v, int o) {
  return cd{__shfl_xor(v.x, o, kWave), __shfl_xor(v.y, o, kWave)};
}

template <typename TY>
__device__ __forceinline__ cd load_c(const TY* p, long long i);
template <>
__device__ __forceinline__ cd load_c<float2>(const float2* p, long long i) {
  const float2 v = p[i];
  return cd{(double)v.x, (double)v.y};
}
template <>
__device__ __forceinline__ cd load_c<double2>(const double2* p, long long i) {
  const double2 v = p[i];
  return cd{v.x, v.y};
}

constexpr int LC = kMaxRankC + 1;
constexpr int TC = 32;  // slab tile edge of the complex tensor pass

__device__ __forceinline__ cd gamma_except_c(const cd* C, int N, int R2, int skip1, int skip2, int e) {
  cd g = cd{1.0, 0.0};
  for (int k = 0; k < N; ++k)
    if (k != skip1 && k != skip2) g = g * C[(long long)k * R2 + e];
  return g;
}

// ---- tensor pass ------------------------------------------------------------

struct PassArgsC {
  const void* Y;
  int I0, I1, N, R;
  long long Q;
  int It[kMaxOrder];
  const cd* A;  // stacked complex factors
  int off[kMaxOrder];
  int tiles_i, tiles_j, q_per;
  cd* m0part;  // [n_qc][tiles_j][R][I0]
  cd* m1part;  // [n_qc][tiles_i][R][I1]
  cd* tpart;   // [tiles_i * tiles_j][R][Q]
  double* e2part;
};

// conj(c_q[r]) = prod_{k >= 3} conj(A^(k)[i_k(q), r])
__device__ cd cq_conj(const PassArgsC& a, long long q, int r) {
  cd c = cd{1.0, 0.0};
  long long qq = q;
  for (int k = 2; k < a.N; ++k) {
    const int Ik = a.It[k - 2];
    const int ik = (int)(qq % Ik);
    qq /= Ik;
    c = c * conjc(a.A[a.off[k] + ik + (long long)r * Ik]);
  }
  return c;
}

// Slab tile 32 x 32 of Y_q on the FP64 matrix cores.  Per slice the three complex products
// of a 32 x 32 tile (Y_hat for the residual, Z_q = Y_q conj(A^(2)) and
// W_q = Y_q^T conj(A^(1))) run as 16 x 16 MFMA tiles, each complex product as
// four real ones (re += a.re b.re - a.im b.im, im += a.re b.im + a.im b.re).
// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16] and B[l/16][l%16] of the
// step and the result D[l/16 + 4v][l%16].  Wave w takes row block w >> 1 and
// column block w & 1 (ranks 16 (w & 1).. of Z and W; columns j of Y_hat).
template <typename TY, bool RESID>
__global__ __launch_bounds__(256) void k_pass_cm(PassArgsC a, const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd Ys[TC][TC + 1];            // Ys[jj][ii] = Y[i0 + ii, j0 + jj, q] (or E)
  __shared__ cd A0s[TC][LC];               // conj(A^(1)) rows of the tile, zero beyond R
  __shared__ cd A1s[TC][LC];               // conj(A^(2)) rows of the tile, zero beyond R
  __shared__ cd A1c[RESID ? TC : 1][LC];   // conj(A^(2)) diag(conj c_q)
  __shared__ cd cq[kMaxRankC];
  __shared__ cd tl[2][kMaxRankC];          // t_q partial of each row block
  __shared__ double red[16];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int R = a.R, I0 = a.I0, I1 = a.I1;
  const int tile = blockIdx.x, tj = tile % a.tiles_j, ti = tile / a.tiles_j;
  const int i0 = ti * TC, j0 = tj * TC;
  const long long q0 = (long long)blockIdx.y * a.q_per;
  long long q1 = q0 + a.q_per;
  if (q1 > a.Q) q1 = a.Q;
  const TY* Y = static_cast<const TY*>(a.Y);
  for (int e = t; e < TC * kMaxRankC; e += 256) {
    const int ii = e % TC, r = e / TC;
    const int gi = i0 + ii, gj = j0 + ii;
    A0s[ii][r] = (r < R && gi < I0) ? conjc(a.A[a.off[0] + gi + (long long)r * I0]) : czero();
    A1s[ii][r] = (r < R && gj < I1) ? conjc(a.A[a.off[1] + gj + (long long)r * I1]) : czero();
  }
  const int xb = w >> 1, rb = w & 1;
  const bool zw_on = rb * 16 < R;
  const int rr = 16 * rb + li;  // rank of this lane's Z and W columns
  cd m0[4], m1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    m0[v] = czero();
    m1[v] = czero();
  }
  double e2 = 0.0;
  cd* tp = a.tpart + (long long)tile * R * a.Q;
  const int KR4 = (R + 3) / 4;
  for (long long q = q0; q < q1; ++q) {
    sync_block();
    if (q > q0 && t < R) tp[(long long)t * a.Q + q - 1] = tl[0][t] + tl[1][t];
    const long long base = (long long)I0 * I1 * q;
    cd yv[TC * TC / 256];
#pragma unroll
    for (int k = 0; k < TC * TC / 256; ++k) {
      const int e = t + 256 * k, ii = e % TC, jj = e / TC;
      const int gi = i0 + ii, gj = j0 + jj;
      yv[k] = (gi < I0 && gj < I1) ? load_c<TY>(Y, base + gi + (long long)I0 * gj) : czero();
    }
    if (t < kMaxRankC) cq[t] = (t < R) ? cq_conj(a, q, t) : czero();
#pragma unroll
    for (int k = 0; k < TC * TC / 256; ++k) {
      const int e = t + 256 * k, ii = e % TC, jj = e / TC;
      Ys[jj][ii] = yv[k];
    }
    sync_block();
    if (RESID) {
      for (int e = t; e < TC * kMaxRankC; e += 256) {
        const int jj = e % TC, r = e / TC;
        A1c[jj][r] = A1s[jj][r] * cq[r];
      }
      sync_block();
      // conj(Y_hat)[i][j] = sum_r A0s[i][r] A1c[j][r]: rows i = 16 xb.., columns j = 16 rb..
      v4d hre = v4d{0.0, 0.0, 0.0, 0.0}, him = v4d{0.0, 0.0, 0.0, 0.0};
      for (int k4 = 0; k4 < KR4; ++k4) {
        const int kk = 4 * k4 + lk;
        const cd av = A0s[16 * xb + li][kk];
        const cd bv = A1c[16 * rb + li][kk];
        hre = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, hre, 0, 0, 0);
        hre = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.y, hre, 0, 0, 0);
        him = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, him, 0, 0, 0);
        him = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, him, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = 16 * xb + lk + 4 * v, jj = 16 * rb + li;
        const cd ev = Ys[jj][ii] - cd{hre[v], -him[v]};  // zero outside the tensor
        e2 += abs2(ev);
        Ys[jj][ii] = ev;
      }
      sync_block();
    }
    if (zw_on) {
      v4d zre = v4d{0.0, 0.0, 0.0, 0.0}, zim = v4d{0.0, 0.0, 0.0, 0.0};
      v4d wre = v4d{0.0, 0.0, 0.0, 0.0}, wim = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < TC / 4; ++k4) {
        const int kk = 4 * k4 + lk;
        // Z: A[i][j] = Y(i, j), i = 16 xb + li, j = kk; B[j][r] = A1s[j][r]
        const cd ya = Ys[kk][16 * xb + li];
        const cd b1 = A1s[kk][rr];
        zre = __builtin_amdgcn_mfma_f64_16x16x4f64(ya.x, b1.x, zre, 0, 0, 0);
        zre = __builtin_amdgcn_mfma_f64_16x16x4f64(-ya.y, b1.y, zre, 0, 0, 0);
        zim = __builtin_amdgcn_mfma_f64_16x16x4f64(ya.x, b1.y, zim, 0, 0, 0);
        zim = __builtin_amdgcn_mfma_f64_16x16x4f64(ya.y, b1.x, zim, 0, 0, 0);
        // W: A[j][i] = Y(i, j), j = 16 xb + li, i = kk; B[i][r] = A0s[i][r]
        const cd yw = Ys[16 * xb + li][kk];
        const cd b0 = A0s[kk][rr];
        wre = __builtin_amdgcn_mfma_f64_16x16x4f64(yw.x, b0.x, wre, 0, 0, 0);
        wre = __builtin_amdgcn_mfma_f64_16x16x4f64(-yw.y, b0.y, wre, 0, 0, 0);
        wim = __builtin_amdgcn_mfma_f64_16x16x4f64(yw.x, b0.y, wim, 0, 0, 0);
        wim = __builtin_amdgcn_mfma_f64_16x16x4f64(yw.y, b0.x, wim, 0, 0, 0);
      }
      const cd c = cq[rr];
      cd tv = czero();
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const cd z = cd{zre[v], zim[v]}, wv = cd{wre[v], wim[v]};
        m0[v] += c * z;
        m1[v] += c * wv;
        tv += A0s[16 * xb + lk + 4 * v][rr] * z;
      }
      // sum over the four row groups of the 16 rows (lanes li + 16 lk)
      tv += shfl_xor_cd(tv, 16);
      tv += shfl_xor_cd(tv, 32);
      if (lk == 0 && rr < R) tl[xb][rr] = tv;
    }
  }
  sync_block();
  if (q1 > q0 && t < R) tp[(long long)t * a.Q + q1 - 1] = tl[0][t] + tl[1][t];
  cd* m0p = a.m0part + ((long long)blockIdx.y * a.tiles_j + tj) * R * I0;
  cd* m1p = a.m1part + ((long long)blockIdx.y * a.tiles_i + ti) * R * I1;
  if (zw_on && rr < R) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ro = 16 * xb + lk + 4 * v;
      if (i0 + ro < I0) m0p[(long long)rr * I0 + i0 + ro] = m0[v];
      if (j0 + ro < I1) m1p[(long long)rr * I1 + j0 + ro] = m1[v];
    }
  }
  if (RESID) {
    const double s = block_sum(e2, red);
    if (t == 0) a.e2part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// dst[x] = sum_s part[s * len + x] (complex), x < len; dst[x] at stride dstride.
__global__ void k_sum_slots_c(const cd* part, int nslots, long long len, cd* dst, const int* stop) {
  if (stopped(stop)) return;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= len) return;
  cd acc = czero();
  for (int s = 0; s < nslots; ++s) acc += part[(long long)s * len + x];
  dst[x] = acc;
}

// Partial buffer [slot][tile][R][I] summed over slots and tiles into M[r * I + i].
__global__ void k_sum_tiles_c(const cd* part, int nslot, int ntile, int R, int I, cd* M, const int* stop) {
  if (stopped(stop)) return;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long len = (long long)R * I;
  if (x >= len) return;
  cd acc = czero();
  for (int s = 0; s < nslot * ntile; ++s) acc += part[(long long)s * len + x];
  M[x] = acc;
}

// Trailing modes k >= 3: M_k[i, r] = sum_{q : i_k(q) = i} t_q[r] prod_{k' != k} conj(A^(k')[i_k'(q), r]).
__global__ void k_modes_from_t_c(PassArgsC a, const cd* tq, cd* M, const int* stop) {
  if (stopped(stop)) return;
  const int R = a.R;
  // flatten (k, i, r) over the trailing modes
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 2; k < a.N; ++k) {
    const int Ik = a.It[k - 2];
    const long long cnt = (long long)Ik * R;
    if (x >= cnt) {
      x -= cnt;
      continue;
    }
    const int i = (int)(x % Ik), r = (int)(x / Ik);
    long long stride = 1;
    for (int kk = 2; kk < k; ++kk) stride *= a.It[kk - 2];
    const long long outer = a.Q / (stride * Ik);
    cd acc = czero();
    for (long long o = 0; o < outer; ++o)
      for (long long in = 0; in < stride; ++in) {
        const long long q = in + stride * ((long long)i + (long long)Ik * o);
        cd c = cd{1.0, 0.0};
        long long qq = q;
        for (int kk = 2; kk < a.N; ++kk) {
          const int I2 = a.It[kk - 2];
          const int ik = (int)(qq % I2);
          qq /= I2;
          if (kk != k) c = c * conjc(a.A[a.off[kk] + ik + (long long)r * I2]);
        }
        acc += tq[(long long)r * a.Q + q] * c;
      }
    M[a.off[k] + i + (long long)r * Ik] = acc;
    return;
  }
}

__global__ void k_sum_e2(const double* part, int n, double* out, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double red[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = acc;
}

// ---- R x R kernels ----------------------------------------------------------

// Partial A^H A over 64-row chunks: part[(n chunks + c) stride + 2e (+1)] (complex), e = r + qR.
__global__ __launch_bounds__(256) void k_gram_part_c(Shape s, const cd* A, double* part, int chunks, int stride,
                                                     const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd As[64][LC];
  const int n = blockIdx.x, c = blockIdx.y, R = s.R, In = s.I[n];
  const int r0 = c * 64;
  cd* out = reinterpret_cast<cd*>(part + ((long long)n * chunks + c) * stride);
  const cd* An = A + (long long)s.off[n] * R;
  for (int e = threadIdx.x; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    As[ii][r] = (r0 + ii < In) ? An[r0 + ii + (long long)r * In] : czero();
  }
  sync_block();
  for (int e = threadIdx.x; e < R * R; e += 256) {
    const int r = e % R, q = e / R;
    cd acc = czero();
    for (int i = 0; i < 64; ++i) acc += conjc(As[i][r]) * As[i][q];
    out[e] = acc;
  }
}

// out[n][x] = sum_c part[(n chunks + c) stride + x], x < len (doubles).
__global__ void k_rows_reduce_c(const double* part, int chunks, int stride, int len, double* out, const int* stop) {
  if (stopped(stop)) return;
  const int n = blockIdx.x;
  for (int x = threadIdx.x; x < len; x += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += part[((long long)n * chunks + c) * stride + x];
    out[(long long)n * len + x] = acc;
  }
}

// Hermitian Cholesky H = L L^H (lower, in place) by one block.  mode 0: a
// non-positive pivot sets *bad.  mode 1 (semidefinite): a pivot below 64 u
// times the original diagonal ref[k] zeroes the column.
__device__ void chol_herm(cd (*H)[LC], int R, int mode, const double* ref, int* bad, cd* lk) {
  const int t = threadIdx.x;
  for (int k = 0; k < R; ++k) {
    sync_block();
    const double dkk = H[k][k].x;
    bool zero = false;
    double inv = 1.0, d = 1.0;
    if (mode == 0) {
      if (!(dkk > 0.0)) {
        if (t == 0) *bad = 1;
      } else {
        d = sqrt(dkk);
        inv = 1.0 / d;
      }
    } else {
      if (!(dkk > 64.0 * 2.220446049250313e-16 * ref[k])) zero = true;
      else {
        d = sqrt(dkk);
        inv = 1.0 / d;
      }
    }
    for (int i = k + t; i < R; i += blockDim.x)
      lk[i] = zero ? czero() : ((i == k) ? cd{d, 0.0} : inv * H[i][k]);
    sync_block();
    for (int e = t; e < R * R; e += blockDim.x) {
      const int i = e % R, j = e / R;
      if (j > k && i >= j) H[i][j] -= lk[i] * conjc(lk[j]);
    }
    for (int i = k + t; i < R; i += blockDim.x) H[i][k] = lk[i];
  }
  sync_block();
  for (int e = t; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    if (j > i) H[i][j] = czero();
  }
  sync_block();
}

// blockIdx.x = n; blockIdx.y = 0: Gamma_n, the Cholesky of Gamma_n + mu I, its
// inverse Li, X_n = Li^H and Gt_n = Li^H Li; blockIdx.y = 1: the semidefinite
// Cholesky L_n of C_n.
__global__ __launch_bounds__(256) void k_gamma_c(Shape s, const cd* C, double mu_host, const FitState* state,
                                                 cd* Gam, cd* Gt, cd* X, cd* Lc, int* bad, const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd H[kMaxRankC][LC];
  __shared__ cd Li[kMaxRankC][LC];
  __shared__ cd lk[kMaxRankC];
  __shared__ double ref[kMaxRankC];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  if (blockIdx.y == 1) {
    for (int e = t; e < R2; e += 256) {
      const int r = e % R, q = e / R;
      H[r][q] = C[(long long)n * R2 + e];
    }
    for (int r = t; r < R; r += 256) ref[r] = C[(long long)n * R2 + r + r * R].x;
    chol_herm(H, R, 1, ref, bad, lk);
    for (int e = t; e < R2; e += 256) {
      const int r = e % R, q = e / R;
      Lc[(long long)n * R2 + e] = H[r][q];
    }
    return;
  }
  const double mu = state ? state->mu : mu_host;
  for (int e = t; e < R2; e += 256) {
    const int r = e % R, q = e / R;
    const cd g = gamma_except_c(C, N, R2, n, -1, e);
    Gam[(long long)n * R2 + e] = g;
    H[r][q] = (r == q) ? cd{g.x + mu, g.y} : g;
  }
  chol_herm(H, R, 0, ref, bad, lk);
  // Li = L^-1, one column per thread: Li[j][j] = 1 / L[j][j], Li[i][j] = -sum_{k=j}^{i-1} L[i][k] Li[k][j] / L[i][i]
  for (int j = t; j < R; j += 256) {
    Li[j][j] = cd{1.0 / H[j][j].x, 0.0};
    for (int i = j + 1; i < R; ++i) {
      cd acc = czero();
      for (int k = j; k < i; ++k) acc += H[i][k] * Li[k][j];
      Li[i][j] = (-1.0 / H[i][i].x) * acc;
    }
    for (int i = 0; i < j; ++i) Li[i][j] = czero();
  }
  sync_block();
  for (int e = t; e < R2; e += 256) {
    const int r = e % R, q = e / R;
    X[(long long)n * R2 + e] = conjc(Li[q][r]);  // X = Li^H
    cd acc = czero();
    for (int k = (r > q ? r : q); k < R; ++k) acc += conjc(Li[k][r]) * Li[k][q];
    Gt[(long long)n * R2 + e] = acc;  // Gt = Li^H Li = (Gamma_n + mu I)^-1
  }
}

// Rows of mode n, chunk c: G = M - A Gamma_n^T (or M when it already is the
// gradient), P = G conj(Gt_n), partial w = A^H P, partial ||G||^2 and ||M||^2.
__global__ __launch_bounds__(256) void k_pw_c(Shape s, const cd* A, const cd* M, int resid, const cd* Gam,
                                              const cd* Gt, cd* Gout, cd* Pout, double* part, int chunks,
                                              int stride, const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd As[64][LC];
  __shared__ cd Gs[64][LC];
  __shared__ cd Ps[64][LC];
  __shared__ cd Gm[kMaxRankC][LC];
  __shared__ double red[16];
  const int n = blockIdx.x, c = blockIdx.y, R = s.R, R2 = R * R, In = s.I[n], t = threadIdx.x;
  const int r0 = c * 64;
  double* outd = part + ((long long)n * chunks + c) * stride;
  cd* out = reinterpret_cast<cd*>(outd);
  if (r0 >= In) {
    for (int e = t; e < 2 * R2 + 4; e += 256) outd[e] = 0.0;
    return;
  }
  const long long base = (long long)s.off[n] * R;
  for (int e = t; e < R2; e += 256) {
    const int r = e % R, q = e / R;
    // Gm[k][r] = Gamma_n^T[k][r] = Gamma_n[r][k] (first product), later conj(Gt)[k][r]
    Gm[q][r] = resid ? conjc(Gt[(long long)n * R2 + q + r * R]) : Gam[(long long)n * R2 + r + q * R];
  }
  double m2 = 0.0;
  for (int e = t; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    const bool ok = r0 + ii < In;
    const long long gi = base + r0 + ii + (long long)r * In;
    As[ii][r] = ok ? A[gi] : czero();
    const cd mv = ok ? M[gi] : czero();
    Gs[ii][r] = mv;
    m2 += abs2(mv);
  }
  sync_block();
  if (!resid) {
    for (int e = t; e < 64 * R; e += 256) {
      const int ii = e & 63, r = e >> 6;
      cd acc = czero();
      for (int k = 0; k < R; ++k) acc += As[ii][k] * Gm[k][r];  // (A Gamma^T)[ii][r]
      Ps[ii][r] = Gs[ii][r] - acc;
    }
    sync_block();
    for (int e = t; e < 64 * R; e += 256) {
      const int ii = e & 63, r = e >> 6;
      Gs[ii][r] = Ps[ii][r];
    }
    for (int e = t; e < R2; e += 256) {
      const int r = e % R, q = e / R;
      Gm[q][r] = conjc(Gt[(long long)n * R2 + q + r * R]);  // conj(Gt)[q][r]
    }
    sync_block();
  }
  double g2 = 0.0;
  for (int e = t; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    cd acc = czero();
    for (int k = 0; k < R; ++k) acc += Gs[ii][k] * Gm[k][r];
    Ps[ii][r] = acc;
    if (r0 + ii < In) {
      const long long gi = base + r0 + ii + (long long)r * In;
      Gout[gi] = Gs[ii][r];
      Pout[gi] = acc;
      g2 += abs2(Gs[ii][r]);
    }
  }
  sync_block();
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd acc = czero();
    for (int i = 0; i < 64; ++i) acc += conjc(As[i][a]) * Ps[i][b];
    out[e] = acc;
  }
  g2 = block_sum(g2, red);
  m2 = block_sum(m2, red);
  if (t == 0) {
    outd[2 * R2 + 0] = g2;
    outd[2 * R2 + 1] = m2;
    outd[2 * R2 + 2] = 0.0;
    outd[2 * R2 + 3] = 0.0;
  }
}

// w_n = sum over row chunks; block 0 also reduces ||G||^2, ||M||^2 into scal[2], scal[3].
__global__ void k_wred_c(Shape s, const double* part, int chunks, int stride, double* w, double* scal,
                         const int* stop) {
  if (stopped(stop)) return;
  const int n = blockIdx.x, R2 = s.R * s.R, N = s.N, t = threadIdx.x;
  for (int e = t; e < 2 * R2; e += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += part[((long long)n * chunks + c) * stride + e];
    w[(long long)n * 2 * R2 + e] = acc;
  }
  if (n == 0 && t < 2) {
    double acc = 0.0;
    for (int m = 0; m < N; ++m)
      for (int c = 0; c < chunks; ++c) acc += part[((long long)m * chunks + c) * stride + 2 * R2 + t];
    scal[2 + t] = acc;
  }
}

// Index of complex entry e of block n in the embedded layout [Re v_1, Im v_1, Re v_t, Im v_t].
__device__ __forceinline__ void emb_index(int n, int e, int R2, int nt, long long* re, long long* im) {
  if (n == 0) {
    *re = e;
    *im = R2 + e;
  } else {
    const long long q = (long long)(n - 1) * R2 + e;
    *re = 2LL * R2 + q;
    *im = 2LL * R2 + nt + q;
  }
}

// z_n = vec(L_n^H V conj(X_n)), V = sum_{m != n} Gamma_nm^T * W_m^T, written embedded.
__global__ __launch_bounds__(256) void k_z_c(Shape s, const cd* C, const cd* w, const cd* X, const cd* Lc,
                                             double* z, const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd V[kMaxRankC][LC];
  __shared__ cd Tm[kMaxRankC][LC];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  const int nt = (N - 1) * R2;
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd v = czero();
    for (int m = 0; m < N; ++m) {
      if (m == n) continue;
      // (Gamma_nm^T * W_m^T)[a][b] = Gamma_nm[b][a] W_m[b][a], W_m[b][a] = w_m[b + aR]
      v += gamma_except_c(C, N, R2, n, m, b + a * R) * w[(long long)m * R2 + b + a * R];
    }
    V[a][b] = v;
  }
  sync_block();
  const cd* L = Lc + (long long)n * R2;
  const cd* Xn = X + (long long)n * R2;
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd acc = czero();
    for (int k = 0; k < R; ++k) acc += conjc(L[k + a * R]) * V[k][b];  // (L^H V)[a][b]
    Tm[a][b] = acc;
  }
  sync_block();
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd acc = czero();
    for (int k = 0; k < R; ++k) acc += Tm[a][k] * conjc(Xn[k + b * R]);
    long long ir, ii;
    emb_index(n, e, R2, nt, &ir, &ii);
    z[ir] = acc.x;
    z[ii] = acc.y;
  }
}

// T_nm[(a + dR) R + j] = sum_i Gamma_nm[j, i] conj(L_n[i, a]) X_m[i, d], n != m.  Grid (N N, R).
__global__ __launch_bounds__(256) void k_tnm_c(Shape s, const cd* C, const cd* X, const cd* Lc, cd* Tnm,
                                               const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd Gs[kMaxRankC][LC];
  __shared__ cd Ls[kMaxRankC][LC];
  __shared__ cd xd[kMaxRankC];
  const int pair = blockIdx.x, d = blockIdx.y, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  const int n = pair / N, m = pair % N;
  if (n == m) return;
  for (int e = t; e < R2; e += 256) {
    const int i = e % R, j = e / R;
    Gs[i][j] = gamma_except_c(C, N, R2, n, m, e);
    Ls[i][j] = conjc(Lc[(long long)n * R2 + e]);
  }
  for (int i = t; i < R; i += 256) xd[i] = X[(long long)m * R2 + i + d * R];
  sync_block();
  cd* out = Tnm + (long long)pair * R * R2;
  for (int e = t; e < R2; e += 256) {
    const int j = e % R, a = e / R;
    cd acc = czero();
    for (int i = 0; i < R; ++i) acc += Gs[j][i] * Ls[i][a] * xd[i];
    out[((long long)a + (long long)d * R) * R + j] = acc;
  }
}

// R x R sub-block (b, d) of S_nm, n > m, written into the real embedding: St for
// m >= 1 (lower triangle of [[Re S, -Im S], [Im S, Re S]] over the trailing
// modes), the embedded block column B for m = 0.
__global__ __launch_bounds__(256) void k_subblock_c(Shape s, SysPlan p, const cd* Tnm, const cd* X, const cd* Lc,
                                                    double* St, double* B, const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd Td[kMaxRankC][LC];  // Td[j][a] = conj(X_n[j, b]) T_nm[j, a + dR]
  __shared__ cd Lm[kMaxRankC][LC];
  const int N = s.N, R = s.R, R2 = R * R, t = threadIdx.x;
  const int nt = (N - 1) * R2;
  int pr = blockIdx.x / R;
  const int b = blockIdx.x % R, d = blockIdx.y;
  int n = 1;
  while (pr >= n) {
    pr -= n;
    ++n;
  }
  const int m = pr;
  const cd* T = Tnm + (long long)(n * N + m) * R * R2;
  for (int e = t; e < R2; e += 256) {
    const int j = e % R, a = e / R;
    Td[j][a] = conjc(X[(long long)n * R2 + j + b * R]) * T[((long long)a + (long long)d * R) * R + j];
    Lm[j][a] = Lc[(long long)m * R2 + e];
  }
  sync_block();
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, c = e / R;
    cd acc = czero();
    for (int j = 0; j < R; ++j) acc += Td[j][a] * Lm[j][c];
    const long long qr = (long long)(n - 1) * R2 + a + b * R;  // complex trailing row
    const long long pc = (long long)c + (long long)d * R;      // column within the block
    if (m == 0) {
      B[qr + pc * p.ntp] = acc.x;
      B[nt + qr + pc * p.ntp] = acc.y;
      B[qr + (R2 + pc) * p.ntp] = -acc.y;
      B[nt + qr + (R2 + pc) * p.ntp] = acc.x;
    } else {
      const long long qc = (long long)(m - 1) * R2 + pc;
      St[qr + qc * p.lds] = acc.x;
      St[nt + qr + (nt + qc) * p.lds] = acc.x;
      St[nt + qr + qc * p.lds] = acc.y;
      St[nt + qc + qr * p.lds] = -acc.y;
    }
  }
}

// u_n = w_n - vec(L_n Y_n X_n^T), Y_n read from the embedded solution.
__global__ __launch_bounds__(256) void k_u_c(Shape s, const cd* w, const double* y, const cd* X, const cd* Lc,
                                             cd* u, const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd Ys[kMaxRankC][LC];
  __shared__ cd Tm[kMaxRankC][LC];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  const int nt = (N - 1) * R2;
  for (int e = t; e < R2; e += 256) {
    long long ir, ii;
    emb_index(n, e, R2, nt, &ir, &ii);
    Ys[e % R][e / R] = cd{y[ir], y[ii]};
  }
  sync_block();
  const cd* L = Lc + (long long)n * R2;
  const cd* Xn = X + (long long)n * R2;
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd acc = czero();
    for (int k = 0; k < R; ++k) acc += L[a + k * R] * Ys[k][b];
    Tm[a][b] = acc;
  }
  sync_block();
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd acc = czero();
    for (int k = 0; k < R; ++k) acc += Tm[a][k] * Xn[b + k * R];  // (Tm X^T)[a][b]
    u[(long long)n * R2 + e] = w[(long long)n * R2 + e] - acc;
  }
}

// F_n = sum_{m != n} Gamma_nm^T * U_m^T (= (K u)_n), Q_n = F_n conj(Gt_n).
__global__ __launch_bounds__(256) void k_fq_c(Shape s, const cd* C, const cd* u, const cd* Gt, cd* f, cd* Q,
                                              const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd Fs[kMaxRankC][LC];
  const int n = blockIdx.x, R = s.R, R2 = R * R, N = s.N, t = threadIdx.x;
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd v = czero();
    for (int m = 0; m < N; ++m) {
      if (m == n) continue;
      v += gamma_except_c(C, N, R2, n, m, b + a * R) * u[(long long)m * R2 + b + a * R];
    }
    f[(long long)n * R2 + e] = v;
    Fs[a][b] = v;
  }
  sync_block();
  const cd* G = Gt + (long long)n * R2;
  for (int e = t; e < R2; e += 256) {
    const int a = e % R, b = e / R;
    cd acc = czero();
    for (int k = 0; k < R; ++k) acc += Fs[a][k] * conjc(G[k + b * R]);
    Q[(long long)n * R2 + e] = acc;
  }
}

// A_c = A + P - A Q_n on the rows of (mode n, chunk c).  Partials: Gram A_c^H A_c,
// sum Re(conj(da) (g + mu da)) and sum |da|^2.
__global__ __launch_bounds__(256) void k_update_c(Shape s, const cd* A, const cd* P, const cd* G, const cd* Q,
                                                  double mu_host, const FitState* state, cd* Ac, double* part,
                                                  int chunks, int stride, cd* da_out, const int* stop) {
  if (stopped(stop)) return;
  __shared__ cd As[64][LC];
  __shared__ cd Qs[kMaxRankC][LC];
  __shared__ cd Cs[64][LC];
  __shared__ double red[16];
  const int n = blockIdx.x, c = blockIdx.y, R = s.R, R2 = R * R, In = s.I[n], t = threadIdx.x;
  const int r0 = c * 64;
  double* outd = part + ((long long)n * chunks + c) * stride;
  cd* out = reinterpret_cast<cd*>(outd);
  if (r0 >= In) {
    for (int e = t; e < 2 * R2 + 4; e += 256) outd[e] = 0.0;
    return;
  }
  const double mu = state ? state->mu : mu_host;
  const long long base = (long long)s.off[n] * R;
  for (int e = t; e < R2; e += 256) Qs[e % R][e / R] = Q[(long long)n * R2 + e];
  for (int e = t; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    As[ii][r] = (r0 + ii < In) ? A[base + r0 + ii + (long long)r * In] : czero();
  }
  sync_block();
  double den = 0.0, da2 = 0.0;
  for (int e = t; e < 64 * R; e += 256) {
    const int ii = e & 63, r = e >> 6;
    cd v = czero();
    if (r0 + ii < In) {
      const long long gi = base + r0 + ii + (long long)r * In;
      cd acc = czero();
      for (int k = 0; k < R; ++k) acc += As[ii][k] * Qs[k][r];
      const cd da = P[gi] - acc;
      v = As[ii][r] + da;
      Ac[gi] = v;
      if (da_out) da_out[gi] = da;
      const cd gm = G[gi] + mu * da;
      den += da.x * gm.x + da.y * gm.y;  // Re(conj(da) (g + mu da))
      da2 += abs2(da);
    }
    Cs[ii][r] = v;
  }
  sync_block();
  for (int e = t; e < R2; e += 256) {
    const int r = e % R, q = e / R;
    cd acc = czero();
    for (int i = 0; i < 64; ++i) acc += conjc(Cs[i][r]) * Cs[i][q];
    out[e] = acc;
  }
  den = block_sum(den, red);
  da2 = block_sum(da2, red);
  if (t == 0) {
    outd[2 * R2 + 0] = den;
    outd[2 * R2 + 1] = da2;
    outd[2 * R2 + 2] = 0.0;
    outd[2 * R2 + 3] = 0.0;
  }
}

__global__ void k_scalars_reduce_c(const double* part, int N, int chunks, int stride, int R2, double* scal,
                                   const int* stop) {
  if (stopped(stop)) return;
  if (threadIdx.x < 2) {
    double acc = 0.0;
    for (int m = 0; m < N; ++m)
      for (int c = 0; c < chunks; ++c) acc += part[((long long)m * chunks + c) * stride + 2 * R2 + threadIdx.x];
    scal[threadIdx.x] = acc;
  }
}

// Re sum_{i,r} conj(A^(1)[i,r]) M_1[i,r] = Re sum y conj(y_hat).
__global__ void k_inner_c(Shape s, const cd* A, const cd* M, double* out) {
  __shared__ double red[16];
  double v = 0.0;
  for (int e = threadIdx.x; e < s.I[0] * s.R; e += blockDim.x) {
    const cd a = A[e], m = M[e];
    v += a.x * m.x + a.y * m.y;
  }
  v = block_sum(v, red);
  if (threadIdx.x == 0) out[0] = v;
}

// ALS update of mode n for complex tensors: A_n = M_n conj(Gt_n) = M_n (Gamma^(n)T)^-1
// (Gt_n = Gamma^(n)^-1, Hermitian; M_n is the MTTKRP on conjugated factors),
// one thread per entry of the column-major I_n x R block.
__global__ __launch_bounds__(256) void k_als_rows_c(Shape s, int n, const cd* M, const cd* Gt, cd* A) {
  __shared__ cd Gs[kMaxRankC * kMaxRankC];
  const int R = s.R, R2 = R * R, In = s.I[n], t = threadIdx.x;
  for (int e = t; e < R2; e += 256) Gs[e] = conjc(Gt[(long long)n * R2 + e]);
  sync_block();
  const cd* Mn = M + (long long)s.off[n] * R;
  cd* An = A + (long long)s.off[n] * R;
  const long long total = (long long)In * R;
  for (long long e = blockIdx.x * 256LL + t; e < total; e += (long long)gridDim.x * 256) {
    const int i = (int)(e % In), r = (int)(e / In);
    cd acc = czero();
    for (int k = 0; k < R; ++k) acc += Mn[i + (long long)k * In] * Gs[k + r * R];
    An[e] = acc;
  }
}

}  // namespace

PassPlan plan_pass_c(const Shape& s) {
  PassPlan p{};
  const int I0 = s.I[0], I1 = s.I[1];
  long long Q = 1;
  for (int n = 2; n < s.N; ++n) Q *= s.I[n];
  p.tiles_i = (I0 + TC - 1) / TC;
  p.tiles_j = (I1 + TC - 1) / TC;
  p.Q = Q;
  const long long tiles = (long long)p.tiles_i * p.tiles_j;
  long long nqc = (1024 + tiles - 1) / tiles;
  if (nqc > Q) nqc = Q;
  if (nqc < 1) nqc = 1;
  p.q_per = (int)((Q + nqc - 1) / nqc);
  p.n_qc = (int)((Q + p.q_per - 1) / p.q_per);
  const size_t R = (size_t)s.R;
  p.m0_elems = 2 * (size_t)p.n_qc * p.tiles_j * R * I0;
  p.m1_elems = 2 * (size_t)p.n_qc * p.tiles_i * R * I1;
  p.t_elems = 2 * (size_t)tiles * R * (size_t)Q;
  p.e2_elems = (size_t)p.n_qc * tiles;
  p.tbuf_elems = s.N >= 4 ? 2 * (size_t)Q * R : 0;
  p.tc_bytes = 8;
  p.mfma = 0;
  return p;
}

// M (stacked complex) = MTTKRP with conjugated factors of Y (resid = false) or of
// E = Y - Y_hat (resid = true; e2out[0] = sum |E|^2).  Y is complex64 or complex128.
hipError_t launch_tensor_pass_c(const Shape& s, bool y64, const void* Y, const double* Ad, bool resid,
                                const PassPlan& p, const PassBuffers& b, double* Md, double* e2out,
                                const int* stop, hipStream_t st) {
  PassArgsC a{};
  a.Y = Y;
  a.I0 = s.I[0];
  a.I1 = s.I[1];
  a.N = s.N;
  a.R = s.R;
  a.Q = p.Q;
  for (int k = 2; k < s.N; ++k) a.It[k - 2] = s.I[k];
  for (int k = 0; k < s.N; ++k) a.off[k] = s.off[k] * s.R;
  a.A = reinterpret_cast<const cd*>(Ad);
  a.tiles_i = p.tiles_i;
  a.tiles_j = p.tiles_j;
  a.q_per = p.q_per;
  a.m0part = reinterpret_cast<cd*>(b.m0part);
  a.m1part = reinterpret_cast<cd*>(b.m1part);
  a.tpart = reinterpret_cast<cd*>(b.tpart);
  a.e2part = b.e2part;
  const dim3 grid((unsigned)(p.tiles_i * p.tiles_j), (unsigned)p.n_qc);
  if (y64) {
    if (resid) k_pass_cm<double2, true><<<grid, 256, 0, st>>>(a, stop);
    else k_pass_cm<double2, false><<<grid, 256, 0, st>>>(a, stop);
  } else {
    if (resid) k_pass_cm<float2, true><<<grid, 256, 0, st>>>(a, stop);
    else k_pass_cm<float2, false><<<grid, 256, 0, st>>>(a, stop);
  }
  cd* M = reinterpret_cast<cd*>(Md);
  const int R = s.R;
  const long long len0 = (long long)R * s.I[0], len1 = (long long)R * s.I[1];
  k_sum_tiles_c<<<(unsigned)((len0 + 255) / 256), 256, 0, st>>>(a.m0part, p.n_qc, p.tiles_j, R, s.I[0],
                                                               M + (long long)s.off[0] * R, stop);
  k_sum_tiles_c<<<(unsigned)((len1 + 255) / 256), 256, 0, st>>>(a.m1part, p.n_qc, p.tiles_i, R, s.I[1],
                                                               M + (long long)s.off[1] * R, stop);
  if (s.N >= 3) {
    const long long lent = (long long)R * p.Q;
    cd* tq = s.N >= 4 ? reinterpret_cast<cd*>(b.tbuf) : M + (long long)s.off[2] * R;
    k_sum_slots_c<<<(unsigned)((lent + 255) / 256), 256, 0, st>>>(a.tpart, p.tiles_i * p.tiles_j, lent, tq, stop);
    if (s.N >= 4) {
      long long cnt = 0;
      for (int k = 2; k < s.N; ++k) cnt += (long long)s.I[k] * R;
      k_modes_from_t_c<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(a, tq, M, stop);
    }
  }
  if (resid && e2out) k_sum_e2<<<1, 256, 0, st>>>(b.e2part, (int)p.e2_elems, e2out, stop);
  return hipGetLastError();
}

hipError_t launch_inner_c(const Shape& s, const double* A, const double* M, double* out, hipStream_t st) {
  k_inner_c<<<1, 256, 0, st>>>(s, reinterpret_cast<const cd*>(A), reinterpret_cast<const cd*>(M), out);
  return hipGetLastError();
}

static inline int part_stride_c(const Shape& s) { return 2 * s.R * s.R + 4; }

hipError_t launch_gram_c(const Shape& s, const double* A, const SmallBuffers& b, double* Cout, const int* stop,
                         hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride_c(s);
  k_gram_part_c<<<dim3(s.N, ch), 256, 0, st>>>(s, reinterpret_cast<const cd*>(A), b.rowpart, ch, stride, stop);
  k_rows_reduce_c<<<s.N, 256, 0, st>>>(b.rowpart, ch, stride, 2 * s.R * s.R, Cout, stop);
  return hipGetLastError();
}

// One trial step of the complex path up to the assembled right-hand side (z) and
// the embedded system blocks (St, B); see the file comment.
hipError_t launch_small_pre_c(const Shape& s, const double* A, const double* M, bool resid, double mu_host,
                              const FitState* state, const SmallBuffers& b, int* singular, const int* stop,
                              hipStream_t st) {
  const int ch = row_chunks(s), stride = part_stride_c(s);
  const cd* C = reinterpret_cast<const cd*>(b.C);
  k_gamma_c<<<dim3(s.N, 2), 256, 0, st>>>(s, C, mu_host, state, reinterpret_cast<cd*>(b.Gam),
                                           reinterpret_cast<cd*>(b.Gt), reinterpret_cast<cd*>(b.X),
                                           reinterpret_cast<cd*>(b.Lc), singular, stop);
  k_pw_c<<<dim3(s.N, ch), 256, 0, st>>>(s, reinterpret_cast<const cd*>(A), reinterpret_cast<const cd*>(M),
                                         resid ? 1 : 0, reinterpret_cast<const cd*>(b.Gam),
                                         reinterpret_cast<const cd*>(b.Gt), reinterpret_cast<cd*>(b.G),
                                         reinterpret_cast<cd*>(b.P), b.wpart, ch, stride, stop);
  k_wred_c<<<s.N, 256, 0, st>>>(s, b.wpart, ch, stride, b.w, b.scal, stop);
  k_z_c<<<s.N, 256, 0, st>>>(s, C, reinterpret_cast<const cd*>(b.w), reinterpret_cast<const cd*>(b.X),
                              reinterpret_cast<const cd*>(b.Lc), b.z, stop);
  k_tnm_c<<<dim3(s.N * s.N, s.R), 256, 0, st>>>(s, C, reinterpret_cast<const cd*>(b.X),
                                                 reinterpret_cast<const cd*>(b.Lc), reinterpret_cast<cd*>(b.Tnm),
                                                 stop);
  return hipGetLastError();
}

hipError_t launch_subblock_c(const Shape& s, const SysPlan& p, const SmallBuffers& b, const SysBuffers& y,
                             const int* stop, hipStream_t st) {
  const int npairs = s.N * (s.N - 1) / 2;
  k_subblock_c<<<dim3(npairs * s.R, s.R), 256, 0, st>>>(s, p, reinterpret_cast<const cd*>(b.Tnm),
                                                         reinterpret_cast<const cd*>(b.X),
                                                         reinterpret_cast<const cd*>(b.Lc), y.St, y.B, stop);
  return hipGetLastError();
}

hipError_t launch_small_post_c(const Shape& s, const double* A, double* Ac, const SmallBuffers& b, double mu_host,
                               const FitState* state, const int* stop, hipStream_t st, double* da_out) {
  const int ch = row_chunks(s), stride = part_stride_c(s);
  k_u_c<<<s.N, 256, 0, st>>>(s, reinterpret_cast<const cd*>(b.w), b.y, reinterpret_cast<const cd*>(b.X),
                              reinterpret_cast<const cd*>(b.Lc), reinterpret_cast<cd*>(b.u), stop);
  k_fq_c<<<s.N, 256, 0, st>>>(s, reinterpret_cast<const cd*>(b.C), reinterpret_cast<const cd*>(b.u),
                               reinterpret_cast<const cd*>(b.Gt), reinterpret_cast<cd*>(b.f),
                               reinterpret_cast<cd*>(b.Q), stop);
  k_update_c<<<dim3(s.N, ch), 256, 0, st>>>(s, reinterpret_cast<const cd*>(A), reinterpret_cast<const cd*>(b.P),
                                             reinterpret_cast<const cd*>(b.G), reinterpret_cast<const cd*>(b.Q),
                                             mu_host, state, reinterpret_cast<cd*>(Ac), b.rowpart, ch, stride,
                                             reinterpret_cast<cd*>(da_out), stop);
  k_rows_reduce_c<<<s.N, 256, 0, st>>>(b.rowpart, ch, stride, 2 * s.R * s.R, b.Cc, stop);
  k_scalars_reduce_c<<<1, 64, 0, st>>>(b.rowpart, s.N, ch, stride, s.R * s.R, b.scal, stop);
  return hipGetLastError();
}

hipError_t launch_gamma_c(const Shape& s, const double* C, double mu_host, const FitState* state,
                          const SmallBuffers& b, int* singular, const int* stop, hipStream_t st) {
  k_gamma_c<<<dim3(s.N, 2), 256, 0, st>>>(s, reinterpret_cast<const cd*>(C), mu_host, state,
                                           reinterpret_cast<cd*>(b.Gam), reinterpret_cast<cd*>(b.Gt),
                                           reinterpret_cast<cd*>(b.X), reinterpret_cast<cd*>(b.Lc), singular, stop);
  return hipGetLastError();
}

hipError_t launch_als_rows_c(const Shape& s, int n, const double* M, const SmallBuffers& b, double* A,
                             hipStream_t st) {
  const long long total = (long long)s.I[n] * s.R;
  long long blocks = (total + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  k_als_rows_c<<<(unsigned)blocks, 256, 0, st>>>(s, n, reinterpret_cast<const cd*>(M),
                                                  reinterpret_cast<const cd*>(b.Gt), reinterpret_cast<cd*>(A));
  return hipGetLastError();
}

}  // namespace dgn
