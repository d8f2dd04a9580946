// Register / LDS building blocks of the FP64 Cholesky on 64 x 64 blocks held
// row-major in LDS (row stride TR): a 16 x 16 L D L^T factorisation by one wave
// with DPP row broadcasts, the row-parallel triangular solve below it, the
// MFMA update of a 16 x 16 block, and the inverse of a 64 x 64 lower factor.
// Used by the NR^2 factorisation (one 64-column panel per phase) and by the
// R x R damped inverses (Gamma_n + mu I)^-1 of Theorem 4.1.
#pragma once
#include "common.hpp"

namespace dgn {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// 1/sqrt(x) to FP64 accuracy: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

constexpr int TR = 66;  // row stride of the panel: T[row][k] MFMA operand reads are bank-conflict free

// Broadcast lane SRC of each 16-lane row of v to that whole row (DPP row_newbcast).
template <int SRC>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + SRC, 0xf, 0xf, true);
}

// 1/x to FP64 accuracy: hardware estimate y = (1 - e)/x refined by one cubic
// step, y (1 + e + e^2) = (1 - e^3)/x.
__device__ __forceinline__ double rcp_f64(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(__builtin_fma(e, e, e), y, y);
}

// Column C of the in-register 16 x 16 factorisation in L D L^T form: lane `row`
// holds row `row` in r.  With a = A[row][C] (unscaled) and d_C = A[C][C], the
// rows below the pivot are updated by A[row][J] -= (a / d_C) A[J][C]; the
// broadcasts of column C do not wait for the reciprocal of the pivot.  r[C]
// keeps a (so lane C keeps d_C).
template <int J>
__device__ __forceinline__ void ldl_update(double (&r)[16], double l, double a) {
  if constexpr (J < 16) {
    r[J] -= l * row_bcast<J>(a);
    ldl_update<J + 1>(r, l, a);
  }
}

// PSD: semidefinite-safe form.  A pivot at or below kPsdTol times the original
// diagonal of its row (ref, one value per lane) ends its column: the column's
// multipliers are zero, and so is the column of the scaled factor.
constexpr double kPsdTol = 64.0 * 2.220446049250313e-16;

// Lanes at or above the pivot row (row <= C) run the same update on their
// entries right of the diagonal; those entries feed no entry on or below it
// (the broadcasts read column C of rows J > C) and ldl_scale clears them.
template <int C, bool PSD>
__device__ __forceinline__ void ldl_column(double (&r)[16], int row, bool& ok, double ref) {
  if constexpr (C < 16) {
    const double a = r[C];
    const double piv = row_bcast<C>(a);
    double l;
    if constexpr (PSD) {
      l = (piv > kPsdTol * row_bcast<C>(ref)) ? a * rcp_f64(piv) : 0.0;
    } else {
      ok = ok && (piv > 0.0);
      l = a * rcp_f64(piv);
    }
    ldl_update<C + 1>(r, l, a);
    ldl_column<C + 1, PSD>(r, row, ok, ref);
  }
}

// Rescale the L D L^T result of one lane to the Cholesky factor:
// L[row][c] = A^(c)[row][c] / sqrt(d_c) (on the diagonal r[c] = d_c, so the
// same product gives sqrt(d_c)), zero right of the diagonal.
template <int C>
__device__ __forceinline__ void ldl_scale(double (&r)[16], int row, double myrsq) {
  if constexpr (C < 16) {
    const double rs = row_bcast<C>(myrsq);
    r[C] = (row >= C) ? r[C] * rs : 0.0;
    ldl_scale<C + 1>(r, row, myrsq);
  }
}

// Cholesky of the 16 x 16 block T[k0.., k0..] by one wave (each 16-lane row of
// the wave computes the same rows).  L goes back into T (zeros above), a
// compact copy into Lkk, and 1/L_cc into rinv[k0 + c].  A non-positive pivot
// sets *bad.  PSD: semidefinite-safe form with the original diagonal in
// dref[k0 + c] (a dropped column gets rinv = 0; *bad is not used).
template <bool PSD = false>
__device__ void chol16(double (*T)[TR], int k0, int* bad, double (*Lkk)[16], double* rinv,
                       const double* dref = nullptr) {
  const int lane = threadIdx.x & 63;
  const int row = lane & 15;
  double r[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) r[j] = T[k0 + row][k0 + j];
  double ref = 0.0;
  if constexpr (PSD) ref = dref[k0 + row];
  bool ok = true;
  ldl_column<0, PSD>(r, row, ok, ref);
  double myd = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (row == j) myd = r[j];
  double myrsq;
  if constexpr (PSD)
    myrsq = (myd > kPsdTol * ref) ? rsqrt_f64(myd) : 0.0;
  else
    myrsq = rsqrt_f64(myd > 0.0 ? myd : 1.0);
  ldl_scale<0>(r, row, myrsq);
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      T[k0 + row][k0 + j] = r[j];
      Lkk[row][j] = r[j];
    }
    rinv[k0 + row] = myrsq;
  }
  if constexpr (!PSD)
    if (!ok && lane == 0) *bad = 1;
}

// Row r of the 16-column block k0: T[r][k0..] <- T[r][k0..] L_kk^-T.
__device__ __forceinline__ void trsm16_row(double (*T)[TR], int r, int k0, const double (*Lkk)[16],
                                           const double* rinv) {
  double x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = T[r][k0 + c];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double v = x[c];
#pragma unroll
    for (int d = 0; d < c; ++d) v -= x[d] * Lkk[c][d];
    x[c] = v * rinv[k0 + c];
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) T[r][k0 + c] = x[c];
}

// T[16 bi.., 16 bj..] -= L_bi L_bj^T over the 16 columns k0.. (one wave):
// A operand T[16 bi + l%16][k0 + k + l/16], B operand T[16 bj + l%16][k0 + k + l/16].
__device__ __forceinline__ void trail16(double (*T)[TR], int bi, int bj, int k0) {
  const int lane = threadIdx.x & 63, cl = lane & 15, kq = lane >> 4;
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 16; k += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[16 * bi + cl][k0 + k + kq], T[16 * bj + cl][k0 + k + kq], acc, 0,
                                               0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) T[16 * bi + kq + 4 * v][16 * bj + cl] -= acc[v];
}

// trail16 on NB blocks (bi[n], bj[n]) at once: every operand read is issued
// first and the blocks' MFMAs interleave, so the wave waits for the LDS and the
// matrix pipeline once instead of once per block.  Each block sums its four
// k-steps in trail16's order (same result bit for bit).  The operands (columns
// k0..k0+15) must lie outside the blocks written (columns right of them).
template <int NB>
__device__ __forceinline__ void trail16_batch(double (*T)[TR], const int (&bi)[NB], const int (&bj)[NB], int k0) {
  const int lane = threadIdx.x & 63, cl = lane & 15, kq = lane >> 4;
  double a[NB][4], b[NB][4];
#pragma unroll
  for (int n = 0; n < NB; ++n)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[n][k] = T[16 * bi[n] + cl][k0 + 4 * k + kq];
      b[n][k] = T[16 * bj[n] + cl][k0 + 4 * k + kq];
    }
  v4d acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < NB; ++n) acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[n][k], b[n][k], acc[n], 0, 0, 0);
#pragma unroll
  for (int n = 0; n < NB; ++n)
#pragma unroll
    for (int v = 0; v < 4; ++v) T[16 * bi[n] + kq + 4 * v][16 * bj[n] + cl] -= acc[n][v];
}

// X = L^-1 for the lower 64 x 64 factor in T rows 0..63, written to X (rows
// 64..127 of the panel array, unused by the diagonal workgroup).  Diagonal
// 16-blocks by forward substitution (wave w inverts block w, lane j a column),
// then the blocks at distance d = 1..3 below the diagonal:
//   X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj.
// Only the leading nb 16-blocks (nb <= 4) are inverted when nb < 4.
__device__ void invert_lower64(double (*T)[TR], double (*X)[TR], const double* rinv, double (*Z)[16][16],
                               int nb = 4) {
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, cl = lane & 15, kq = lane >> 4;
  if (w < nb) {
    const int b0 = 16 * w, j = cl;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) v -= T[b0 + i][b0 + k] * x[k];
      x[i] = v * rinv[b0 + i];
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) X[b0 + i][b0 + j] = x[i];
    }
  }
  sync_block();
  for (int d = 1; d < nb; ++d) {
    const int j = w, i = w + d;
    if (i < nb) {
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      for (int k = j; k < i; ++k)
#pragma unroll
        for (int s2 = 0; s2 < 16; s2 += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[16 * i + cl][16 * k + s2 + kq], X[16 * k + s2 + kq][16 * j + cl],
                                                     acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) Z[w][kq + 4 * v][cl] = acc[v];
      // Z is written and read by the same wave only
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s2 = 0; s2 < 16; s2 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[16 * i + cl][16 * i + s2 + kq], Z[w][s2 + kq][cl], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[16 * i + kq + 4 * v][16 * j + cl] = -acc[v];
    }
    sync_block();
  }
}

}  // namespace

}  // namespace dgn
