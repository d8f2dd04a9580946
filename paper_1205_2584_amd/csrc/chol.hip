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
// backward substitution is carried along the phases as Gauss-Jordan
// elimination on the factor (systems of up to 48 tiles) or runs tile by tile
// afterwards (larger systems).
#include "common.hpp"
#include "internal.hpp"
#include "panel.hpp"

namespace dgn {

namespace {

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

// Stage a 64 x 64 column-major global tile into LDS as T[col][row]
// (coalesced; all 16 loads of a thread are issued before the LDS stores).
__device__ __forceinline__ void stage(double (*T)[TL], const double* g, long long ld) {
  double v[16];
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
    v[s2] = g[r + (long long)c * ld];
  }
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
    T[c][r] = v[s2];
  }
}

// Same, stored row-major: T[row][col].
__device__ __forceinline__ void stage_rowmajor(double (*T)[TL], const double* g, long long ld) {
  double v[16];
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
    v[s2] = g[r + (long long)c * ld];
  }
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
    T[r][c] = v[s2];
  }
}

// acc[blk] += A * B^T from LDS tiles stored [col][row]; wave w owns rows
// 16w.. of A; the result element (v, blk) is (A B^T)[acc_row(v)][acc_col(blk)].
__device__ __forceinline__ void mma_lds(const double (*A)[TL], const double (*B)[TL], v4d acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ra = 16 * w + (lane & 15), kk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < 64; k += 4) {
    const double a = A[k + kk][ra];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
      acc[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[k + kk][16 * blk + (lane & 15)], acc[blk], 0, 0, 0);
  }
}

// ---- panel factorisation helpers ----------------------------------------------
//
// The panel of phase ph is the stacked 128 x 64 block [D; B] (D the diagonal
// tile, B one tile below it) held row-major in LDS with row stride TR.  It is
// factored in four 16-column steps: a 16 x 16 Cholesky of the diagonal block by
// one wave, a row-parallel triangular solve for every row below it, and an MFMA
// update of the columns to its right.

// Stage a 64 x 64 column-major global tile into LDS rows T[r][c] (row stride TR).
__device__ __forceinline__ void stage_panel(double (*T)[TR], const double* g, long long ld) {
  double v[16];
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
    v[s2] = g[r + (long long)c * ld];
  }
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
    T[r][c] = v[s2];
  }
}

// Blocks of the in-panel update after column step kb: the lower blocks of D to
// the right of it, then the blocks of B in those columns.
__device__ __forceinline__ void panel_trail_block(int b, int kb, int& bi, int& bj) {
  const int m = 3 - kb, ndb = m * (m + 1) / 2;
  if (b < ndb) {
    bi = (b >= 1) + (b >= 3);
    bj = b - bi * (bi + 1) / 2;
    bi += kb + 1;
    bj += kb + 1;
  } else {
    bi = 4 + (b - ndb) / m;
    bj = kb + 1 + (b - ndb) % m;
  }
}

// The lower blocks of D right of column step KB, by the chain wave in one batch.
template <int KB>
__device__ __forceinline__ void trail_diag(double (*T)[TR]) {
  constexpr int m = 3 - KB, NB = m * (m + 1) / 2;
  int bi[NB], bj[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) panel_trail_block(b, KB, bi[b], bj[b]);
  trail16_batch<NB>(T, bi, bj, 16 * KB);
}

// The blocks of B right of column step KB in the row blocks rb0..rb0+NRB-1
// that one B wave owns, in one batch.
template <int KB, int NRB>
__device__ __forceinline__ void trail_rows(double (*T)[TR], int rb0) {
  constexpr int m = 3 - KB, NB = NRB * m;
  int bi[NB], bj[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    bi[b] = rb0 + b / m;
    bj[b] = KB + 1 + b % m;
  }
  trail16_batch<NB>(T, bi, bj, 16 * KB);
}

// id < ntri: lower tile id (ti, tj) of St (identity / zeros), or a tile of the
// right-hand-side row (zeros); id >= ntri: one of the nbz blocks that zero B.
// skip_sub: leave out the positions k_subblock writes (the off-diagonal mode
// blocks of St and the first R^2 columns of B's first nt rows), so that both
// can run in one launch.
__device__ void fill_body(const SysPlan& p, double* St, double* B, int R2p, long long id, long long nbz,
                          int skip_sub) {
  const long long ntri = (long long)p.Tt * (p.Tt + 1) / 2 + p.Tt;  // lower tiles + RHS row tiles
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
      if (skip_sub && ti < p.Tt && r < p.nt && c < p.nt && r / p.R2 > c / p.R2) continue;
      double v = 0.0;
      if (ti < p.Tt && r == c) v = 1.0;
      St[r + (long long)c * p.lds] = v;
    }
  } else {
    const long long nb = (long long)p.ntp * R2p;
    for (long long e = (id - ntri) * 256 + threadIdx.x; e < nb; e += nbz * 256) {
      if (skip_sub && e % p.ntp < p.nt && e / p.ntp < p.R2) continue;
      B[e] = 0.0;
    }
  }
}

// Fill the lower tiles of St and all of B with identity / zeros (the
// off-diagonal blocks are overwritten by the sub-block kernel afterwards).
__global__ __launch_bounds__(256) void k_fill(SysPlan p, double* St, double* B, int R2p,
                                              const int* stop) {
  if (stopped(stop)) return;
  const long long ntri = (long long)p.Tt * (p.Tt + 1) / 2 + p.Tt;
  fill_body(p, St, B, R2p, blockIdx.x, (long long)gridDim.x - ntri, 0);
}

// R x R sub-block (b, d) of S_nm for n > m: rows n R^2 + a + b R, columns m R^2 + c + d R.
// RM: the rank bound the LDS tiles are sized for (32 or 64), so that ranks up to
// 32 keep several blocks per CU.
// One launch: blocks [0, npairs R^2) form the sub-blocks ((pair, b) fastest,
// then d); the blocks after them run fill_body with the positions written here
// left out (nbz of them zero B).
template <int RM>
__global__ __launch_bounds__(256) void k_subblock(Shape s, SysPlan p, const double* Tnm,
                                                  const double* X, const double* Lc, double* St,
                                                  double* B, int R2p, long long nbz, int write_b,
                                                  const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Td[RM][RM + 1];  // Td[i][a] = T_nm[i, a + dR]
  __shared__ double Lm[RM][RM + 1];
  const int N = s.N, R = s.R, R2 = R * R;
  const long long nx = (long long)(N * (N - 1) / 2) * R, nsub = nx * R;
  if ((long long)blockIdx.x >= nsub) {
    fill_body(p, St, B, R2p, (long long)blockIdx.x - nsub, nbz, 1);
    return;
  }
  const int bx = (int)(blockIdx.x % nx), by = (int)(blockIdx.x / nx);
  // decode the strictly lower pair (n, m), n > m
  int pr = bx / R, b = bx % R, d = by;
  int n = 1, m = 0;
  while (pr >= n) { pr -= n; ++n; }
  m = pr;
  // the block column B (m = 0) only where a dense product still reads it
  if (m == 0 && !write_b) return;
  const int pair = n * N + m;
  const double* T = Tnm + (long long)pair * R * R2;
  {
    // all loads of the thread in flight at once; x_b folded into T on the way to LDS:
    // Td[i][a] = x_b[i] T_nm[i, a + dR], Lm[i][c] = L_m[i, c]
    constexpr int NS = RM * RM / 256;  // entries per thread
    const int i = threadIdx.x & (RM - 1), a0 = threadIdx.x / RM;
    const bool iok = i < R;
    double tv[NS], lv[NS];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const int a = a0 + (256 / RM) * s2;
      const bool ok = iok && a < R;
      tv[s2] = ok ? T[((long long)a + (long long)d * R) * R + i] : 0.0;
      lv[s2] = ok ? Lc[(long long)m * R2 + i + a * R] : 0.0;
    }
    const double xbi = iok ? X[(long long)n * R2 + i + b * R] : 0.0;
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const int a = a0 + (256 / RM) * s2;
      if (iok && a < R) {
        Td[i][a] = tv[s2] * xbi;
        Lm[i][a] = lv[s2];
      }
    }
  }
  sync_block();
  const int sh = R <= 16 ? 4 : (R <= 32 ? 5 : 6);
  const int a = threadIdx.x & ((1 << sh) - 1), cg = threadIdx.x >> sh, cstep = 256 >> sh;
  if (a < R) {
    const long long row = (long long)(n - 1) * R2 + a + b * R;  // trailing row index
    for (int c0 = cg; c0 < R; c0 += 4 * cstep) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = 0; i < R; ++i) {
        const double ta = Td[i][a];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u * cstep;
          if (c < R) acc[u] += ta * Lm[i][c];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * cstep;
        if (c >= R) continue;
        if (m == 0) {
          B[row + (long long)(c + d * R) * p.ntp] = acc[u];
        } else {
          const long long col = (long long)(m - 1) * R2 + c + d * R;
          St[row + col * p.lds] = acc[u];
        }
      }
    }
  }
}

// Right-hand side row: St[ntp, q] = z_t[q] - (B z_1)[q]; 64 rows per block,
// the R^2 sum split over the block's four waves (four partial sums each).
__device__ __forceinline__ void rhs_block(const SysPlan& p, const double* B, const double* z, double* St,
                                          int blk) {
  __shared__ double part[4][65];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int q = blk * 64 + lane;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (q < p.nt) {
    int k = g;
    for (; k + 12 < p.R2; k += 16) {
      a0 += B[q + (long long)k * p.ntp] * z[k];
      a1 += B[q + (long long)(k + 4) * p.ntp] * z[k + 4];
      a2 += B[q + (long long)(k + 8) * p.ntp] * z[k + 8];
      a3 += B[q + (long long)(k + 12) * p.ntp] * z[k + 12];
    }
    for (; k < p.R2; k += 4) a0 += B[q + (long long)k * p.ntp] * z[k];
  }
  part[g][lane] = (a0 + a1) + (a2 + a3);
  sync_block();
  if (g == 0 && q < p.ntp) {
    const double acc = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    St[p.ntp + (long long)q * p.lds] = (q < p.nt) ? z[p.R2 + q] - acc : 0.0;
  }
}

__device__ __forceinline__ void tri_index(long long id, int& ti, int& tj) {
  ti = (int)((sqrt(8.0 * id + 1.0) - 1.0) / 2.0);
  while ((long long)(ti + 1) * (ti + 2) / 2 <= id) ++ti;
  while ((long long)ti * (ti + 1) / 2 > id) --ti;
  tj = (int)(id - (long long)ti * (ti + 1) / 2);
}

// St_tt -= B B^T on the lower tiles; K = R^2 in chunks of KC staged through LDS.
// acc[blk] += A * B^T from LDS tiles stored [k][row] with row stride 80 (the
// [k][row] MFMA operand reads are then bank-conflict free); wave w owns rows
// 16w.. of A.
constexpr int TS = 80;
// Summation chunk of the SYRK: 48 rows of k, so that the two staged operand
// tiles take 60 KB of LDS and two workgroups fit on a CU.
constexpr int KC = 48;
__device__ __forceinline__ void mma_lds80(const double (*A)[TS], const double (*B)[TS], v4d acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ra = 16 * w + (lane & 15), kk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < KC; k += 4) {
    const double a = A[k + kk][ra];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
      acc[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[k + kk][16 * blk + (lane & 15)], acc[blk], 0, 0, 0);
  }
}

// S_tt -= B B^T on the lower tiles (ti >= tj).  The KC-wide chunks of the
// summation range are double-buffered in registers: the next chunk is in
// flight while the current one runs on MFMA.  The first ntp / 64 blocks form
// the right-hand-side row instead, which no tile block touches.
__global__ __launch_bounds__(256) void k_syrk(SysPlan p, const double* B, const double* z, int R2p,
                                              double* St, const int* stop) {
  if (stopped(stop)) return;
  const int nrhs = p.ntp / 64;
  if ((int)blockIdx.x < nrhs) {  // the right-hand-side row, independent of the tiles below
    rhs_block(p, B, z, St, blockIdx.x);
    return;
  }
  __shared__ double Ti[KC][TS];
  __shared__ double Tj[KC][TS];
  int ti, tj;
  tri_index((long long)blockIdx.x - nrhs, ti, tj);
  v4d acc[4];
  zero_acc(acc);
  constexpr int NS = KC / 4;  // elements of a chunk per thread
  double vi[NS], vj[NS];
  auto load = [&](int k0) {
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
      const bool ok = k0 + c < R2p;
      vi[s2] = ok ? B[ti * 64 + r + (long long)(k0 + c) * p.ntp] : 0.0;
      vj[s2] = ok ? B[tj * 64 + r + (long long)(k0 + c) * p.ntp] : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < R2p; k0 += KC) {
    sync_block();
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const int e = threadIdx.x + 256 * s2, r = e & 63, c = e >> 6;
      Ti[c][r] = vi[s2];
      Tj[c][r] = vj[s2];
    }
    sync_block();
    if (k0 + KC < R2p) load(k0 + KC);
    mma_lds80(Tj, Ti, acc);
  }
  double* C = St + ti * 64 + (long long)tj * 64 * p.lds;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk)
#pragma unroll
    for (int v = 0; v < 4; ++v) C[acc_col(blk) + (long long)acc_row(v) * p.lds] -= acc[blk][v];
}

// ---- the Schur update from the structure of B (R <= 32) ----------------------
//
// The eliminated block column is B = [S_21; S_31; ...] with
//   S_n1[a + bR, c + dR] = sum_i X_n[i,b] L_1[i,c] T_n1[i, a + dR].
// Summing over c (C' = L_1 L_1^T) and d first, its Gram blocks are
//   (S_n1 S_q1^T)[a + bR, a' + b'R]
//     = sum_{i,i'} X_n[i,b] X_q[i',b'] C'[i,i'] sum_d T_n1[i, a + dR] T_q1[i', a' + dR],
// that is X_n^T (C' o (T_a T_a'^T)) X_q for each (a, a'), with T_a[i][d] =
// T_n1[i, a + dR]: 3 R^5 multiply-adds per block pair against the R^6 of the
// dense product B B^T.  One workgroup takes a block pair (n, q), q <= n, one a'
// and kBbtAG values of a; each R x R product runs as 16 x 16 FP64 MFMA tiles (R
// padded to 16 or 32, one output tile per wave).  Within a diagonal block pair
// only the entries in tiles on or below the diagonal are updated, as by the
// dense product.  The last (N - 1) R + 1 blocks form the right-hand-side row.
constexpr int kBbtAG = 4;
constexpr int BL = 33;  // leading dimension of the 32 x 32 LDS operands

// One 16 x 16 MFMA tile of an R x R product with K (16 or 32) a compile-time
// constant: every LDS operand of the chain is read before the first MFMA.
// a(k) / b(k): this lane's A / B operand for the k-step starting at k.
template <int KK, typename FA, typename FB>
__device__ __forceinline__ v4d mfma_chain(FA a, FB b) {
  double av[KK / 4], bv[KK / 4];
#pragma unroll
  for (int s2 = 0; s2 < KK / 4; ++s2) {
    av[s2] = a(4 * s2);
    bv[s2] = b(4 * s2);
  }
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s2 = 0; s2 < KK / 4; ++s2) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s2], bv[s2], acc, 0, 0, 0);
  return acc;
}
template <typename FA, typename FB>
__device__ __forceinline__ v4d mfma_chain_k(int K, FA a, FB b) {
  return K == 32 ? mfma_chain<32>(a, b) : mfma_chain<16>(a, b);
}

__global__ __launch_bounds__(256, 2) void k_bbt(Shape s, SysPlan p, const double* z, const double* Tnm,
                                                const double* X, const double* Lc, double* St, const int* stop) {
  if (stopped(stop)) return;
  const int R = s.R, R2 = R * R, N = s.N, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int ng = (R + kBbtAG - 1) / kBbtAG;
  // Workgroups go to the 8 XCDs in turn: block b = 8 k + x runs on XCD x.  All
  // a-groups of one column group (block pair, a') share an XCD, so that the
  // 128-byte lines of St they update together, and T_q, meet in one L2.
  const long long ncg = (long long)(N - 1) * N / 2 * R, ntb = 8 * ((ncg + 7) / 8) * ng;
  __shared__ double Tq[32][BL];  // T_q1[i', a' + dR] as [i'][d]
  __shared__ double Xn[32][BL];
  __shared__ double Xq[32][BL];
  __shared__ double TW[32][BL];  // T_a, then W = X_n^T V
  __shared__ double UV[32][BL];  // L_1 (for C'), then V = C' o U
  // X_n^T V X_q of the group's values of a: rows padded to BL and the slices
  // staggered by 8 doubles, so that neither the MFMA stores nor the column reads
  // of the write-out meet in one LDS bank
  constexpr int OS = 32 * BL + 8;
  __shared__ double Out[kBbtAG * OS];
  const int cl = lane & 15, kq = lane >> 4;
  const int nt = (R + 15) >> 4, K = 16 * nt;
  if ((long long)blockIdx.x >= ntb) {
    // the right-hand-side row z_t - B z_1 from the same structure:
    //   (S_n1 z_1)[a + bR] = sum_i X_n[i,b] Q[i,a],  Q[i,a] = sum_d T_n1[i, a + dR] P[i,d],
    // P = L_1 Z_1.  Block (n, a) forms Q[:, a] and the R rows a + bR of mode n; the
    // last block zeroes the padding.
    const long long rid = (long long)blockIdx.x - ntb;
    if (rid == (long long)(N - 1) * R) {
      for (int x = p.nt + t; x < p.ntp; x += 256) St[p.ntp + (long long)x * p.lds] = 0.0;
      return;
    }
    const int n = (int)(rid / R) + 1, a = (int)(rid % R);
    const double* Tn = Tnm + (long long)(n * N) * R * R2;
    double (*Zs)[BL] = Tq;
    double (*Ls)[BL] = Xq;
    double (*Ps)[BL] = TW;
    double (*Ts)[BL] = UV;  // Ts[i][d] = T_n1[i, a + dR]
    double* Qv = &Out[0];
    {
      double vz[4], vl[4], vx[4], vt[4];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int e = t + 256 * s2, r = e & 31, c2 = e >> 5;
        const bool ok = r < R && c2 < R;
        vz[s2] = ok ? z[r + c2 * R] : 0.0;  // Z_1[c][d] = z_1[c + dR]
        vl[s2] = ok ? Lc[r + c2 * R] : 0.0;
        vx[s2] = ok ? X[(long long)n * R2 + r + c2 * R] : 0.0;
        vt[s2] = ok ? Tn[(long long)(a + c2 * R) * R + r] : 0.0;
      }
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int e = t + 256 * s2, r = e & 31, c2 = e >> 5;
        Zs[r][c2] = vz[s2];
        Ls[r][c2] = vl[s2];
        Xn[r][c2] = vx[s2];
        Ts[r][c2] = vt[s2];
      }
    }
    sync_block();
    if (w < nt * nt) {  // P = L_1 Z_1 (all K columns, zero beyond R)
      const int ti = w % nt, tj = w / nt;
      const v4d acc = mfma_chain_k(
          K, [&](int k) { return Ls[16 * ti + cl][k + kq]; }, [&](int k) { return Zs[k + kq][16 * tj + cl]; });
#pragma unroll
      for (int v = 0; v < 4; ++v) Ps[16 * ti + kq + 4 * v][16 * tj + cl] = acc[v];
    }
    sync_block();
    if (t < R) {  // Q[i][a] = sum_d Ts[i][d] P[i][d]
      double acc = 0.0;
      for (int d = 0; d < R; ++d) acc += Ts[t][d] * Ps[t][d];
      Qv[t] = acc;
    }
    sync_block();
    if (t < R) {  // row a + tR: z_n[a + tR] - sum_i X_n[i][t] Q[i]
      double acc = 0.0;
      for (int i = 0; i < R; ++i) acc += Xn[i][t] * Qv[i];
      const int e = a + t * R;
      St[p.ntp + ((long long)(n - 1) * R2 + e) * p.lds] = z[(long long)n * R2 + e] - acc;
    }
    return;
  }
  const long long kx = (long long)blockIdx.x / 8, cgi = (kx / ng) * 8 + blockIdx.x % 8;
  if (cgi >= ncg) return;
  const int grp = (int)(kx % ng);
  const int ap = (int)(cgi % R);
  int pr = (int)(cgi / R);
  int n = 1;
  while (pr >= n) {
    pr -= n;
    ++n;
  }
  const int q = pr + 1;
  const double* Tn = Tnm + (long long)(n * N) * R * R2;  // T_n1: pair (n, mode 1)
  const double* Tqg = Tnm + (long long)(q * N) * R * R2;
  // wave w < nt^2 owns output tile (ti, tj) of every product
  const bool tw = w < nt * nt;
  const int ti = w % nt, tj = w / nt;
  const int a0 = grp * kBbtAG, na = (R - a0 < kBbtAG) ? R - a0 : kBbtAG;
  // Every global load of the block at once: the operands, the kBbtAG slices
  // T_a and the St entries it updates (no other block writes them).  St[(n-1)
  // R^2 + a + bR, (q-1) R^2 + a' + b'R]: wave w takes the columns b' = w, w + 4,
  // ..., its lanes the rows (a, b) with the group's values of a adjacent.
  const long long rb = (long long)(n - 1) * R2 + a0, cb = (long long)(q - 1) * R2 + ap;
  constexpr int NW = 16;  // 8 columns x 2 row halves per lane
  long long gi[NW];
  double old[NW];
  double vq[4], vn[4], vx[4], vl[4], tv[kBbtAG][4];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    const int e = t + 256 * s2, r = e & 31, c2 = e >> 5;
    const bool ok = r < R && c2 < R;
    vq[s2] = ok ? Tqg[(long long)(ap + c2 * R) * R + r] : 0.0;
    vn[s2] = ok ? X[(long long)n * R2 + r + c2 * R] : 0.0;
    vx[s2] = ok ? X[(long long)q * R2 + r + c2 * R] : 0.0;
    vl[s2] = ok ? Lc[r + c2 * R] : 0.0;  // L_1
#pragma unroll
    for (int al = 0; al < kBbtAG; ++al)
      tv[al][s2] = (ok && al < na) ? Tn[(long long)(a0 + al + c2 * R) * R + r] : 0.0;
  }
#pragma unroll
  for (int s2 = 0; s2 < NW; ++s2) {
    const int bq = w + 4 * (s2 >> 1), idx = lane + 64 * (s2 & 1), al = idx & (kBbtAG - 1), b = idx / kBbtAG;
    const long long r = rb + al + (long long)b * R, c2 = cb + (long long)bq * R;
    const bool ok = bq < R && b < R && al < na && !(n == q && (r >> 6) < (c2 >> 6));
    gi[s2] = ok ? r + c2 * p.lds : -1;
    old[s2] = ok ? St[gi[s2]] : 0.0;
  }
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    const int e = t + 256 * s2, r = e & 31, c2 = e >> 5;
    Tq[r][c2] = vq[s2];
    Xn[r][c2] = vn[s2];
    Xq[r][c2] = vx[s2];
    UV[r][c2] = vl[s2];
  }
  sync_block();
  // C' = L_1 L_1^T on this wave's tile, kept in registers
  v4d c1 = v4d{0.0, 0.0, 0.0, 0.0};
  if (tw)
    c1 = mfma_chain_k(
        K, [&](int k) { return UV[16 * ti + cl][k + kq]; }, [&](int k) { return UV[16 * tj + cl][k + kq]; });
  sync_block();
#pragma unroll
  for (int al = 0; al < kBbtAG; ++al) {
    if (al >= na) break;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int e = t + 256 * s2, r = e & 31, c2 = e >> 5;
      TW[r][c2] = tv[al][s2];
    }
    sync_block();
    if (tw) {
      // U = T_a T_q^T, V = C' o U
      const v4d acc = mfma_chain_k(
          K, [&](int k) { return TW[16 * ti + cl][k + kq]; }, [&](int k) { return Tq[16 * tj + cl][k + kq]; });
#pragma unroll
      for (int v = 0; v < 4; ++v) UV[16 * ti + kq + 4 * v][16 * tj + cl] = c1[v] * acc[v];
    }
    sync_block();
    if (tw) {
      // W = X_n^T V
      const v4d acc = mfma_chain_k(
          K, [&](int k) { return Xn[k + kq][16 * ti + cl]; }, [&](int k) { return UV[k + kq][16 * tj + cl]; });
#pragma unroll
      for (int v = 0; v < 4; ++v) TW[16 * ti + kq + 4 * v][16 * tj + cl] = acc[v];
    }
    sync_block();
    if (tw) {
      // X_n^T V X_q
      const v4d acc = mfma_chain_k(
          K, [&](int k) { return TW[16 * ti + cl][k + kq]; }, [&](int k) { return Xq[k + kq][16 * tj + cl]; });
#pragma unroll
      for (int v = 0; v < 4; ++v) Out[al * OS + (16 * ti + kq + 4 * v) * BL + 16 * tj + cl] = acc[v];
    }
    sync_block();
  }
#pragma unroll
  for (int s2 = 0; s2 < NW; ++s2) {
    const int bq = w + 4 * (s2 >> 1), idx = lane + 64 * (s2 & 1), al = idx & (kBbtAG - 1), b = idx / kBbtAG;
    if (gi[s2] >= 0) St[gi[s2]] = old[s2] - Out[al * OS + b * BL + bq];
  }
}

// y_1 = z_1 - B^T y_t from the structure of B (R <= 32):
//   (B^T y_t)[c + dR] = sum_i L_1[i,c] H[i,d],
//   H[i,d] = sum_{n >= 2} sum_a T_n1[i, a + dR] G_n[i,a],  G_n = X_n Y_n^T, Y_n[a][b] = y_n[a + bR].
// Block d forms H[:, d] and the entries c + dR (each block also copies part of
// y_t into y).
__global__ __launch_bounds__(256) void k_y0s(Shape s, SysPlan p, const double* z, const double* yt,
                                             const double* Tnm, const double* X, const double* Lc, double* y,
                                             const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Xs[32][BL];
  __shared__ double Ys[32][BL];
  __shared__ double Gs[32][BL];
  __shared__ double Hp[8][32];
  __shared__ double Hv[32];
  const int R = s.R, R2 = R * R, N = s.N, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int cl = lane & 15, kq = lane >> 4, nt = (R + 15) >> 4, K = 16 * nt;
  const int d = blockIdx.x;
  const int i = t & 31, ac = t >> 5;  // H: row i, values of a ac, ac + 8, ...
  double h = 0.0;
  for (int n = 1; n < N; ++n) {
    const double* Tn = Tnm + (long long)(n * N) * R * R2;
    double vx[4], vy[4], tv[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int e = t + 256 * s2, r = e & 31, c2 = e >> 5;
      const bool ok = r < R && c2 < R;
      vx[s2] = ok ? X[(long long)n * R2 + r + c2 * R] : 0.0;
      vy[s2] = ok ? yt[(long long)(n - 1) * R2 + r + c2 * R] : 0.0;  // Y_n[r][c2]
      const int a = ac + 8 * s2;
      tv[s2] = (i < R && a < R) ? Tn[(long long)(a + d * R) * R + i] : 0.0;
    }
    sync_block();  // the previous mode's G is no longer read
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int e = t + 256 * s2, r = e & 31, c2 = e >> 5;
      Xs[r][c2] = vx[s2];
      Ys[r][c2] = vy[s2];
    }
    sync_block();
    if (w < nt * nt) {  // G = X_n Y_n^T
      const int ti = w % nt, tj = w / nt;
      const v4d acc = mfma_chain_k(
          K, [&](int k) { return Xs[16 * ti + cl][k + kq]; }, [&](int k) { return Ys[16 * tj + cl][k + kq]; });
#pragma unroll
      for (int v = 0; v < 4; ++v) Gs[16 * ti + kq + 4 * v][16 * tj + cl] = acc[v];
    }
    sync_block();
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int a = ac + 8 * s2;
      if (i < R && a < R) h += tv[s2] * Gs[i][a];
    }
  }
  Hp[ac][i] = h;
  sync_block();
  if (t < 32) {
    double acc = 0.0;
#pragma unroll
    for (int g = 0; g < 8; ++g) acc += Hp[g][t];
    Hv[t] = acc;
  }
  sync_block();
  if (t < R) {  // entry c = t: z_1[c + dR] - sum_i L_1[i][c] H[i]
    double acc = 0.0;
    for (int i2 = 0; i2 < R; ++i2) acc += Lc[i2 + t * R] * Hv[i2];
    y[t + d * R] = z[t + d * R] - acc;
  }
  for (int q = blockIdx.x * 256 + t; q < p.nt; q += gridDim.x * 256) y[p.R2 + q] = yt[q];
}

// Phase ph of the tiled Cholesky.  Blocks [0, Tt - ph + 1) are the panel row
// tiles i = ph + blk (the last one is the right-hand-side row).  Each applies
// the update of column ph-1 to the diagonal tile D and to its tile B, then
// factors [D; B] in LDS.  Block 0 (i = ph, no B) writes L(ph, ph) to Ld.  Every diagonal-tile copy is read from St,
// which this launch never writes.  The remaining blocks are the trailing tiles
// (i, j), ph < j <= i <= Tt, j < Tt, which receive the update of column ph-1.
// Their MFMA operands load straight from global memory into registers.  The
// launches reserve LDS so that each workgroup has its CU alone
// (phase_lds_reserve).
// Bounded wait until the workgroup-shared counter reaches `target`; on
// exhaustion (never expected: the waves waited on make progress on their own)
// the singular flag is raised and the wait ends.
__device__ __forceinline__ void wait_at_least(int* ctr, int target, int* bad) {
  int spins = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > (1 << 22)) {
      if ((threadIdx.x & 63) == 0) *bad = 1;
      return;
    }
  }
}

// Barrier of waves 1..3 (wave 0 runs the diagonal chain meanwhile).
__device__ __forceinline__ void barrier3(int* ctr, int& epoch, int* bad) {
  ++epoch;
  if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  wait_at_least(ctr, 3 * epoch, bad);
}

// ---- solution by Gauss-Jordan elimination on the factor --------------------------
//
// The backward substitution y_k = L_kk^-T (w_k - sum_{m > k} L_mk^T y_m) (w the
// forward-substituted right-hand side, which rides along the factorisation) is
// carried along the phases instead of after them.  Step s (tile column s
// factored) writes a_s = L_ss^-T w_s and G_sm = L_ss^-T L_ms^T (m > s), so that
// y_s = a_s - sum_{m > s} G_sm y_m; step s then eliminates y_s from every
// earlier relation: a_k -= G_ks a_s and G_km -= G_ks G_sm (k < s < m).  After
// the last step y_k = a_k.  G_km lives in the upper tile (k, m) of St, which the
// factorisation never touches, and a in yt.  The launch of phase ph writes step
// ph - 1 and eliminates with step ph - 2, so every operand comes from an earlier
// launch; these blocks run beside the panel of phase ph and are off its critical
// path.  Two launches after the last phase finish the elimination.
__host__ __device__ inline int phase_panels(const SysPlan& p, int ph) { return ph < p.Tt ? p.Tt - ph + 1 : 0; }
__host__ __device__ inline long long phase_trailing(const SysPlan& p, int ph) {
  if (ph <= 0 || ph >= p.Tt) return 0;
  long long n = 0;
  for (int j = ph + 1; j < p.Tt; ++j) n += p.Tt - j + 1;
  return n;
}
// Tiles of a row per block (measured at 500^3, R = 30: one tile per block keeps
// the phases shortest; three per block made them 0.4 us longer on average).
constexpr int kGjGroup = 1;
// The elimination does about Tt^3 / 6 tile products, as many flops as the
// factorisation itself; it pays while a phase's elimination blocks (up to
// (Tt / 2)^2) fit beside the panel in one round of the CUs.  Larger systems
// (the explicit dGN Hessian, R > 45) take the tile-by-tile backward
// substitution after the factorisation instead.
constexpr int kGjMaxTiles = 48;
__host__ __device__ inline bool use_gj(const SysPlan& p) { return p.Tt <= kGjMaxTiles; }
__host__ __device__ inline int gj_groups(const SysPlan& p, int s) { return (p.Tt - 1 - s + kGjGroup - 1) / kGjGroup; }
// write blocks of step s: groups of the tiles G_sm, m in (s, Tt - 1], then the vector a_s
__host__ __device__ inline long long gj_writes(const SysPlan& p, int s) {
  return (use_gj(p) && s >= 0 && s < p.Tt) ? gj_groups(p, s) + 1 : 0;
}
// elimination blocks of step s: groups of the tiles (k, m), k < s < m < Tt, then the vectors a_k, k < s
__host__ __device__ inline long long gj_elims(const SysPlan& p, int s) {
  return (use_gj(p) && s >= 0 && s < p.Tt) ? (long long)s * gj_groups(p, s) + s : 0;
}
__host__ inline long long phase_blocks(const SysPlan& p, int ph) {
  return phase_panels(p, ph) + phase_trailing(p, ph) + gj_writes(p, ph - 1) + gj_elims(p, ph - 2);
}

// X = L_ss^-1 (rows 64..127 of T) from the factored diagonal tile Ld[s].
__device__ void gj_inverse(const SysPlan& p, const double* Ld, int s, double (*T)[TR], double* rinv,
                           double (*Z)[16][16]) {
  stage_panel(T, Ld + (long long)s * 64 * 64, 64);
  // invert_lower64 writes the lower blocks of X only: the blocks above the
  // diagonal start at zero, since the products below sum over whole rows
  for (int e = threadIdx.x; e < 64 * 64; e += 256) T[64 + (e >> 6)][e & 63] = 0.0;
  sync_block();
  if (threadIdx.x < 64) rinv[threadIdx.x] = 1.0 / T[threadIdx.x][threadIdx.x];
  sync_block();
  invert_lower64(T, T + 64, rinv, Z);
  sync_block();
}

// The blocks reuse the phase kernel's LDS: T (128 x TR), rinv (64) and the
// 4 x 16 x 16 panel array Lk (the inversion's scratch); the partial sums of the
// vector blocks go to the first 256 doubles of T once T's first rows are free.
__device__ void gj_block(const SysPlan& p, int ph, double* St, const double* Ld, double* yt, long long id,
                         double (*T)[TR], double* rinv, double (*Z)[16][16]) {
  double* vec = rinv;
  double (*part)[64] = reinterpret_cast<double (*)[64]>(&T[0][0]);
  const long long lds = p.lds;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, cl = lane & 15, kq = lane >> 4;
  const int sw = ph - 1, se = ph - 2;
  const long long nw = gj_writes(p, sw);
  if (id < nw) {
    // step sw: G_sw,m = (L(m, sw) X)^T, or the vector a_sw = X^T w_sw
    gj_inverse(p, Ld, sw, T, rinv, Z);
    const double (*X)[TR] = T + 64;
    if (id == nw - 1) {
      if (t < 64) vec[t] = St[p.ntp + (long long)(64 * sw + t) * lds];
      sync_block();
      // a[c] = sum_r X[r][c] w[r]; wave g sums r = g, g + 4, ...
      double acc = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2) {
        const int r = w + 4 * s2;
        acc += X[r][lane] * vec[r];
      }
      part[w][lane] = acc;
      sync_block();
      if (t < 64) yt[64 * sw + t] = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
      return;
    }
    const int m0 = sw + 1 + kGjGroup * (int)id;
    const int m1 = m0 + kGjGroup < p.Tt ? m0 + kGjGroup : p.Tt;
    for (int m = m0; m < m1; ++m) {
      const double* A = St + 64 * m + (long long)(64 * sw) * lds;  // L(m, sw), column-major
      // P = A X: wave w forms rows 16w.. of P; lane: A[16w + cl][k0 + kq], X[k0 + kq][16 blk + cl]
      double av[16];
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2) av[s2] = A[(16 * w + cl) + (long long)(4 * s2 + kq) * lds];
      v4d acc[4];
      zero_acc(acc);
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2)
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
          acc[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s2], X[4 * s2 + kq][16 * blk + cl], acc[blk], 0, 0, 0);
      // acc[blk][v] = P[16w + kq + 4v][16blk + cl] = G[16blk + cl][16w + kq + 4v]
      double* G = St + 64 * sw + (long long)(64 * m) * lds;
#pragma unroll
      for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int v = 0; v < 4; ++v) G[(16 * blk + cl) + (long long)(16 * w + kq + 4 * v) * lds] = acc[blk][v];
    }
    return;
  }
  id -= nw;
  // elimination with step se (its G_se,m and a_se were written by the previous launch)
  const int ngrp = gj_groups(p, se);
  const long long ntile = (long long)se * ngrp;
  if (id < ntile) {
    const int k = (int)(id / ngrp), m0 = se + 1 + kGjGroup * (int)(id % ngrp);
    const int m1 = m0 + kGjGroup < p.Tt ? m0 + kGjGroup : p.Tt;
    // C = G_ks G_sm computed as C^T: A-operand G_sm^T[c][j] = TB[j][c], B-operand G_ks^T[j][r] = TA[j][r];
    // G_ks is staged once for the group
    const double* Gks = St + 64 * k + (long long)(64 * se) * lds;  // column-major
    double (*TA)[TR] = T;       // TA[j][r] = G_ks(r, j)
    double (*TB)[TR] = T + 64;  // TB[j][c] = G_sm(j, c)
    for (int m = m0; m < m1; ++m) {
      const double* Gsm = St + 64 * se + (long long)(64 * m) * lds;
      double* Gkm = St + 64 * k + (long long)(64 * m) * lds;
      double va[16], vb[16];
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2) {
        const int e = t + 256 * s2, r = e & 63, c = e >> 6;
        if (m == m0) va[s2] = Gks[r + (long long)c * lds];
        vb[s2] = Gsm[r + (long long)c * lds];
      }
      if (m > m0) sync_block();  // the previous tile's products have read TB
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2) {
        const int e = t + 256 * s2, r = e & 63, c = e >> 6;
        if (m == m0) TA[c][r] = va[s2];
        TB[r][c] = vb[s2];
      }
      sync_block();
      v4d acc[4];
      zero_acc(acc);
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2) {
        const double a = TB[4 * s2 + kq][16 * w + cl];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
          acc[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, TA[4 * s2 + kq][16 * blk + cl], acc[blk], 0, 0, 0);
      }
      // acc[blk][v] = C^T[16w + kq + 4v][16blk + cl] = C[16blk + cl][16w + kq + 4v]
#pragma unroll
      for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int v = 0; v < 4; ++v) Gkm[(16 * blk + cl) + (long long)(16 * w + kq + 4 * v) * lds] -= acc[blk][v];
    }
    return;
  }
  id -= ntile;
  // a_k -= G_k,se a_se
  const int k = (int)id;
  const double* Gks = St + 64 * k + (long long)(64 * se) * lds;
  if (t < 64) vec[t] = yt[64 * se + t];
  double g[16];
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) g[s2] = Gks[lane + (long long)(w + 4 * s2) * lds];
  sync_block();
  double acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) acc += g[s2] * vec[w + 4 * s2];
  part[w][lane] = acc;
  sync_block();
  if (t < 64) yt[64 * k + t] -= (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
}

__global__ __launch_bounds__(256, 2) void k_chol_phase(SysPlan p, int ph, double* St, double* Ld,
                                                       double* yt, int* bad, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double T[128][TR];
  __shared__ __align__(16) double Lk[4][16][16];  // L_kk of each column step
  __shared__ double rinv[64];
  __shared__ int step_done, b_count, d_done;
  const int npanel = phase_panels(p, ph);
  const long long lds = p.lds;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int cl = lane & 15, kq = lane >> 4;
  if ((int)blockIdx.x < npanel) {
    // the panel is the critical path of the phase
    __builtin_amdgcn_s_setprio(3);
    const int i = ph + blockIdx.x;
    const bool hb = (i != ph);
    const double* Dg = St + ph * 64 + (long long)ph * 64 * lds;
    double* Bg = St + i * 64 + (long long)ph * 64 * lds;
    if (t == 0) {
      step_done = 0;
      b_count = 0;
      d_done = 0;
    }
    const double* La = St + ph * 64 + (long long)(ph - 1) * 64 * lds;  // L(ph, ph-1) (ph > 0)
    const double* Lb = St + i * 64 + (long long)(ph - 1) * 64 * lds;   // L(i, ph-1)
    // Update of column ph-1 by row blocks: wave w takes D row block dri (column
    // blocks 0..dri) and then its B row blocks.  The column operand (all of
    // L(ph, ph-1)) is read once per half of the summation range.
    auto load_half = [&](int h, int bi, int ncol, const double* P, double (&av)[8], double (&bv)[4][8]) {
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) {
        const long long ko = (long long)(32 * h + 4 * s2 + kq) * lds;
        av[s2] = P[((bi & 3) * 16 + cl) + ko];
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q][s2] = (q < ncol) ? La[(16 * q + cl) + ko] : 0.0;
      }
    };
    auto mfma_half = [&](const double (&av)[8], const double (&bv)[4][8], int ncol, v4d (&acc)[4]) {
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < ncol) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s2], bv[q][s2], acc[q], 0, 0, 0);
    };
    auto update_rows = [&](int bi, int ncol, const double* P, const double (&av0)[8], const double (&bv0)[4][8]) {
      // av0 / bv0: the first half, already loaded
      v4d acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
      double av1[8], bv1[4][8];
      load_half(1, bi, ncol, P, av1, bv1);
      mfma_half(av0, bv0, ncol, acc);
      mfma_half(av1, bv1, ncol, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < ncol)
#pragma unroll
          for (int v = 0; v < 4; ++v) T[16 * bi + kq + 4 * v][16 * q + cl] -= acc[q][v];
    };
    const int dri = (w == 0) ? 0 : 4 - w;  // D row block of this wave: 0, 3, 2, 1
    double av0[8], bv0[4][8];
    if (ph > 0) load_half(0, dri, dri + 1, La, av0, bv0);  // in flight while the panel is staged
    stage_panel(T, Dg, lds);
    if (hb) stage_panel(T + 64, Bg, lds);
    sync_block();
    if (ph > 0) update_rows(dri, dri + 1, La, av0, bv0);
    if (lane == 0) __hip_atomic_fetch_add(&d_done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (w == 0) {
      // Diagonal chain: factor D step by step.  After the rows of D below the
      // diagonal block of step kb are solved, publish kb + 1.
      for (int kb = 0; kb < 4; ++kb) {
        const int k0 = 16 * kb;
        chol16(T, k0, bad, Lk[kb], rinv);
        // D(0, 0) is this wave's own row block; the rest of D must be updated
        // before the first solve and update below
        if (kb == 0) wait_at_least(&d_done, 4, bad);
        if (lane < 48 - k0) trsm16_row(T, k0 + 16 + lane, k0, Lk[kb], rinv);
        if (lane == 0) __hip_atomic_store(&step_done, kb + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (kb == 0)
          trail_diag<0>(T);
        else if (kb == 1)
          trail_diag<1>(T);
        else if (kb == 2)
          trail_diag<2>(T);
      }
    } else if (hb) {
      // Waves 1..3: the rows of B.  Update with column ph-1, then follow the chain.
      int epoch = 0;
      if (ph > 0) {
        load_half(0, 4 + (w - 1), 4, Lb, av0, bv0);
        update_rows(4 + (w - 1), 4, Lb, av0, bv0);  // B row blocks 4, 5, 6 ...
        if (w == 3) {                              // ... and 7
          load_half(0, 7, 4, Lb, av0, bv0);
          update_rows(7, 4, Lb, av0, bv0);
        }
      }
      barrier3(&b_count, epoch, bad);
      // From here on each B wave owns whole row blocks (wave 1 row blocks 4 and
      // 5, waves 2 and 3 row blocks 6 and 7): its solves and its updates touch
      // only its own rows, so the steps wait for the chain's progress only.
      // Between them, the fence orders the LDS hand-off among the wave's lanes.
      const int rb0 = (w == 1) ? 4 : w + 4, nrows = (w == 1) ? 32 : 16;
      for (int kb = 0; kb < 4; ++kb) {
        const int k0 = 16 * kb;
        wait_at_least(&step_done, kb + 1, bad);
        if (lane < nrows) trsm16_row(T, 16 * rb0 + lane, k0, Lk[kb], rinv);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (w == 1) {
          if (kb == 0)
            trail_rows<0, 2>(T, 4);
          else if (kb == 1)
            trail_rows<1, 2>(T, 4);
          else if (kb == 2)
            trail_rows<2, 2>(T, 4);
        } else {
          if (kb == 0)
            trail_rows<0, 1>(T, rb0);
          else if (kb == 1)
            trail_rows<1, 1>(T, rb0);
          else if (kb == 2)
            trail_rows<2, 1>(T, rb0);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
      }
    }
    sync_block();
    if (!hb) {
      double* Lg = Ld + (long long)ph * 64 * 64;
      for (int e = t; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        Lg[r + c * 64] = (c <= r) ? T[r][c] : 0.0;
      }
    } else {
      for (int e = t; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        Bg[r + c * lds] = T[64 + r][c];
      }
    }
    return;
  }
  long long id = (long long)blockIdx.x - npanel;
  const long long nupd = phase_trailing(p, ph);
  if (id >= nupd) {
    gj_block(p, ph, St, Ld, yt, id - nupd, T, rinv, Lk);
    return;
  }
  int j = ph + 1;
  while (id >= (long long)(p.Tt - j + 1)) {
    id -= (p.Tt - j + 1);
    ++j;
  }
  const int i = j + (int)id;
  // C(i, j) -= L(i, ph-1) L(j, ph-1)^T, computed in 16-column strips of C^T:
  // wave w forms (L(j) L(i)^T)[16w.., :] = C[:, 16w..]^T.
  const double* Ltj = St + j * 64 + (long long)(ph - 1) * 64 * lds;
  const double* Lti = St + i * 64 + (long long)(ph - 1) * 64 * lds;
  double* C = St + i * 64 + (long long)j * 64 * lds;
  v4d acc[4];
  zero_acc(acc);
  for (int h = 0; h < 2; ++h) {  // two halves of k, operands loaded ahead of each half
    double av[8], bv[4][8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const long long ko = (long long)(32 * h + 4 * s2 + kq) * lds;
      av[s2] = Ltj[(16 * w + cl) + ko];
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) bv[blk][s2] = Lti[(16 * blk + cl) + ko];
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) acc[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s2], bv[blk][s2], acc[blk], 0, 0, 0);
  }
  // acc[blk][v] = (L(j) L(i)^T)[16w + kq + 4v][16blk + cl] = C[16blk + cl][16w + kq + 4v]
#pragma unroll
  for (int blk = 0; blk < 4; ++blk)
#pragma unroll
    for (int v = 0; v < 4; ++v) C[(16 * blk + cl) + (long long)(16 * w + kq + 4 * v) * lds] -= acc[blk][v];
}

// L_kk^-1 of every diagonal tile (row-major, into Li), one workgroup per tile,
// after the factorisation: the inverses only serve the backward substitution.
__global__ __launch_bounds__(256) void k_inv_diag(SysPlan p, const double* Ld, double* Li, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double T[64][TR];
  __shared__ double X[64][TR];
  __shared__ double rinv[64];
  __shared__ double Z[4][16][16];
  const int k = blockIdx.x, t = threadIdx.x;
  stage_panel(T, Ld + (long long)k * 64 * 64, 64);
  sync_block();
  if (t < 64) rinv[t] = 1.0 / T[t][t];
  sync_block();
  invert_lower64(T, X, rinv, Z);
  double* Xg = Li + (long long)k * 64 * 64;
  for (int e = t; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    Xg[c + r * 64] = (c <= r) ? X[r][c] : 0.0;
  }
}

// Backward substitution, phase k (descending).  Every block forms
// y_k = L_kk^-T u_k from the inverse tile (u_k is the right-hand-side row of
// tile column k); block k stores y_k and block j < k updates u_j -= L_kj^T y_k.
__global__ __launch_bounds__(256) void k_bsolve(SysPlan p, int k, double* St, const double* Li, double* yt,
                                                const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Lt[64][TL];  // staged L(k, j), [col][row]
  __shared__ double u[64];
  __shared__ double ys[64];
  __shared__ double part[4][64];
  const long long lds = p.lds;
  const int t = threadIdx.x, j = blockIdx.x, c = t & 63, g = t >> 6;
  if (t < 64) u[t] = St[p.ntp + (long long)(k * 64 + t) * lds];
  if (j != k) stage(Lt, St + k * 64 + (long long)j * 64 * lds, lds);
  sync_block();
  // y_k[c] = sum_r X[r][c] u[r], X = L_kk^-1 stored row-major
  const double* X = Li + (long long)k * 64 * 64;
  double acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int r = g + 4 * s2;
    acc += X[r * 64 + c] * u[r];
  }
  part[g][c] = acc;
  sync_block();
  if (t < 64) ys[t] = part[0][t] + part[1][t] + part[2][t] + part[3][t];
  sync_block();
  if (j == k) {
    if (t < 64) yt[k * 64 + t] = ys[t];
    return;
  }
  // u_j[c] -= sum_r L(k, j)[r][c] y_k[r]
  acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int r = g + 4 * s2;
    acc += Lt[c][r] * ys[r];
  }
  part[g][c] = acc;
  sync_block();
  if (t < 64) {
    const double v = part[0][t] + part[1][t] + part[2][t] + part[3][t];
    St[p.ntp + (long long)(j * 64 + t) * lds] -= v;
  }
}

// Backward substitution for the tile pair (k, k-1), k >= 1 (descending).  Every
// block forms y_k = L_kk^-T u_k, u'_{k-1} = u_{k-1} - L(k, k-1)^T y_k and
// y_{k-1} = L_{k-1,k-1}^-T u'_{k-1} from the inverse tiles; blocks k and k-1
// store them, block j < k-1 updates u_j -= L(k, j)^T y_k + L(k-1, j)^T y_{k-1}.
// All loads of a thread are issued before the first product.
__global__ __launch_bounds__(256) void k_bsolve2(SysPlan p, int k, double* St, const double* Li, double* yt,
                                                 const int* stop) {
  if (stopped(stop)) return;
  __shared__ double Lt[3][64][TL];  // L(k, k-1), L(k, j), L(k-1, j), each [col][row]
  __shared__ double u[2][64];
  __shared__ double ys[2][64];
  __shared__ double part[4][64];
  const long long lds = p.lds;
  const int t = threadIdx.x, j = blockIdx.x, c = t & 63, g = t >> 6;
  const bool upd = j < k - 1;
  const double* src[3] = {St + k * 64 + (long long)(k - 1) * 64 * lds, upd ? St + k * 64 + (long long)j * 64 * lds : nullptr,
                          upd ? St + (k - 1) * 64 + (long long)j * 64 * lds : nullptr};
  const double* Xk = Li + (long long)k * 64 * 64;          // L_kk^-1, row-major
  const double* Xk1 = Li + (long long)(k - 1) * 64 * 64;
  double v[3][16], xk[16], xk1[16], u0 = 0.0, u1 = 0.0;
  if (t < 64) {
    u0 = St[p.ntp + (long long)(k * 64 + t) * lds];
    u1 = St[p.ntp + (long long)((k - 1) * 64 + t) * lds];
  }
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int r = g + 4 * s2;
    xk[s2] = Xk[r * 64 + c];
    xk1[s2] = Xk1[r * 64 + c];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
      const int e = t + 256 * s2, rr = e & 63, cc = e >> 6;
      v[m][s2] = src[m] ? src[m][rr + (long long)cc * lds] : 0.0;
    }
  if (t < 64) {
    u[0][t] = u0;
    u[1][t] = u1;
  }
#pragma unroll
  for (int m = 0; m < 3; ++m)
    if (src[m])
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2) {
        const int e = t + 256 * s2, rr = e & 63, cc = e >> 6;
        Lt[m][cc][rr] = v[m][s2];
      }
  sync_block();
  // y_k[c] = sum_r X_k[r][c] u_k[r]
  double acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) acc += xk[s2] * u[0][g + 4 * s2];
  part[g][c] = acc;
  sync_block();
  if (t < 64) ys[0][t] = part[0][t] + part[1][t] + part[2][t] + part[3][t];
  sync_block();
  // u_{k-1}[c] -= sum_r L(k, k-1)[r][c] y_k[r]
  acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int r = g + 4 * s2;
    acc += Lt[0][c][r] * ys[0][r];
  }
  part[g][c] = acc;
  sync_block();
  if (t < 64) u[1][t] -= part[0][t] + part[1][t] + part[2][t] + part[3][t];
  sync_block();
  // y_{k-1}[c] = sum_r X_{k-1}[r][c] u'_{k-1}[r]
  acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) acc += xk1[s2] * u[1][g + 4 * s2];
  part[g][c] = acc;
  sync_block();
  if (t < 64) ys[1][t] = part[0][t] + part[1][t] + part[2][t] + part[3][t];
  sync_block();
  if (j >= k - 1) {
    if (t < 64) yt[(long long)j * 64 + t] = ys[j == k ? 0 : 1][t];
    return;
  }
  // u_j[c] -= sum_r L(k, j)[r][c] y_k[r] + L(k-1, j)[r][c] y_{k-1}[r]
  acc = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int r = g + 4 * s2;
    acc += Lt[1][c][r] * ys[0][r] + Lt[2][c][r] * ys[1][r];
  }
  part[g][c] = acc;
  sync_block();
  if (t < 64) {
    const double d = part[0][t] + part[1][t] + part[2][t] + part[3][t];
    St[p.ntp + (long long)(j * 64 + t) * lds] -= d;
  }
}

// y_1 = z_1 - B^T y_t (one wave per entry) and y[R^2 + q] = y_t[q].
__global__ __launch_bounds__(256) void k_y0(SysPlan p, const double* B, const double* z,
                                            const double* yt, double* y, const int* stop) {
  if (stopped(stop)) return;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k < p.R2) {
    // four independent partial sums, so that four loads per lane are in flight
    const double* Bk = B + (long long)k * p.ntp;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int q = lane;
    for (; q + 192 < p.nt; q += 256) {
      a0 += Bk[q] * yt[q];
      a1 += Bk[q + 64] * yt[q + 64];
      a2 += Bk[q + 128] * yt[q + 128];
      a3 += Bk[q + 192] * yt[q + 192];
    }
    for (; q < p.nt; q += 64) a0 += Bk[q] * yt[q];
    const double acc = wave_sum((a0 + a1) + (a2 + a3));
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
  const long long nsub = (long long)(s.N * (s.N - 1) / 2) * s.R * s.R;
  // R <= 32: the Schur update, the right-hand side and y_1 come from the structure
  // of B, which is then neither written nor cleared
  const bool dense_b = s.R > 32;
  const long long extra = dense_b ? (nbblocks < 1024 ? nbblocks : 1024) : 0;
  const unsigned nblk = (unsigned)(nsub + ntri + extra);
  if (s.R <= 32)
    k_subblock<32><<<nblk, 256, 0, st>>>(s, p, b.Tnm, b.X, b.Lc, y.St, y.B, R2p, extra, dense_b ? 1 : 0, stop);
  else
    k_subblock<64><<<nblk, 256, 0, st>>>(s, p, b.Tnm, b.X, b.Lc, y.St, y.B, R2p, extra, 1, stop);
  if (s.R <= 32) {
    // B B^T from the structure of B (3 R^5 per block pair instead of the dense (N-1)^2 R^6)
    const long long ncg = (long long)(s.N - 1) * s.N / 2 * s.R;
    const long long ntb = 8 * ((ncg + 7) / 8) * ((s.R + kBbtAG - 1) / kBbtAG);
    k_bbt<<<(unsigned)(ntb + (long long)(s.N - 1) * s.R + 1), 256, 0, st>>>(s, p, b.z, b.Tnm, b.X, b.Lc, y.St,
                                                                                 stop);
  } else {
    k_syrk<<<(unsigned)(p.ntp / 64 + (long long)p.Tt * (p.Tt + 1) / 2), 256, 0, st>>>(p, y.B, b.z, R2p, y.St, stop);
  }
  return hipGetLastError();
}

hipError_t launch_sys_fill(const SysPlan& p, const SysBuffers& y, const int* stop, hipStream_t st) {
  const int R2p = r2pad(p.R2);
  const long long ntri = (long long)p.Tt * (p.Tt + 1) / 2 + p.Tt;
  const long long nbblocks = ((long long)p.ntp * R2p + 255) / 256;
  long long extra = nbblocks < 1024 ? nbblocks : 1024;
  k_fill<<<(unsigned)(ntri + extra), 256, 0, st>>>(p, y.St, y.B, R2p, stop);
  return hipGetLastError();
}

hipError_t launch_sys_rhs_syrk(const SysPlan& p, const double* z, const SysBuffers& y, const int* stop,
                               hipStream_t st) {
  const int R2p = r2pad(p.R2);
  k_syrk<<<(unsigned)(p.ntp / 64 + (long long)p.Tt * (p.Tt + 1) / 2), 256, 0, st>>>(p, y.B, z, R2p, y.St, stop);
  return hipGetLastError();
}

SysPlan plan_sys_c(const Shape& s) {
  SysPlan p{};
  p.R2 = 2 * s.R * s.R;
  p.nt = 2 * (s.N - 1) * s.R * s.R;
  p.ntp = ((p.nt + 63) / 64) * 64;
  p.Tt = p.ntp / 64;
  p.lds = p.ntp + 64;
  return p;
}

// Dynamic LDS reserved by a phase launch on top of the kernel's own, so that a
// workgroup takes more than half of a CU's 160 KB and has its CU alone.  It
// pays where the phase is latency-bound, its blocks fitting in about two
// rounds of the CUs: measured at 500^3, R = 30 (at most 463 blocks a phase),
// two workgroups per CU let the trailing and elimination blocks' FP64 MFMA
// slow the panel's FP64 VALU chain (0.710 ms of phases per trial against 0.665
// ms with one per CU).  Phases with more blocks are bound by the trailing
// update and keep two per CU (with every phase exclusive, the explicit dGN
// step at R = 30, 141 tiles, went from 16.2 to 25.4 ms).  The kernel keeps the
// register budget of two workgroups per CU (its launch bounds), which
// scheduled faster than the budget of one (0.670 ms).
constexpr long long kExclusiveMaxBlocks = 512;
static unsigned phase_lds_reserve(long long nblocks) {
  static const unsigned v = [] {
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_chol_phase)) != hipSuccess) return 8192u;
    const size_t half = 160 * 1024 / 2;
    return a.sharedSizeBytes > half ? 0u : (unsigned)(half - a.sharedSizeBytes + 1024);
  }();
  return nblocks <= kExclusiveMaxBlocks ? v : 0u;
}

hipError_t launch_sys_factor_solve_core(const SysPlan& p, const SysBuffers& y, int* singular, const int* stop,
                                        hipStream_t st) {
  if (use_gj(p)) {
    // Tt factorisation phases (each also writing and eliminating the solution's
    // Gauss-Jordan steps), then two launches that finish the elimination
    for (int ph = 0; ph < p.Tt + 2; ++ph) {
      const long long nb = phase_blocks(p, ph);
      if (nb > 0) k_chol_phase<<<(unsigned)nb, 256, phase_lds_reserve(nb), st>>>(p, ph, y.St, y.Ld, y.yt, singular, stop);
    }
    return hipGetLastError();
  }
  // large systems: the factorisation, every L_kk^-1, then the backward
  // substitution two tiles per launch
  for (int ph = 0; ph < p.Tt; ++ph) {
    const long long nb = phase_blocks(p, ph);
    k_chol_phase<<<(unsigned)nb, 256, phase_lds_reserve(nb), st>>>(p, ph, y.St, y.Ld, y.yt, singular, stop);
  }
  k_inv_diag<<<p.Tt, 256, 0, st>>>(p, y.Ld, y.Li, stop);
  int k = p.Tt - 1;
  for (; k >= 1; k -= 2) k_bsolve2<<<k + 1, 256, 0, st>>>(p, k, y.St, y.Li, y.yt, stop);
  if (k == 0) k_bsolve<<<1, 256, 0, st>>>(p, 0, y.St, y.Li, y.yt, stop);
  return hipGetLastError();
}

hipError_t launch_sys_factor_solve(const Shape& s, const SysPlan& p, const SmallBuffers& b,
                                   const SysBuffers& y, int* singular, const int* stop,
                                   hipStream_t st, bool structured_b) {
  hipError_t e = launch_sys_factor_solve_core(p, y, singular, stop, st);
  if (e != hipSuccess) return e;
  if (structured_b)
    k_y0s<<<s.R, 256, 0, st>>>(s, p, b.z, y.yt, b.Tnm, b.X, b.Lc, b.y, stop);
  else
    k_y0<<<(p.R2 + 3) / 4, 256, 0, st>>>(p, y.B, b.z, y.yt, b.y, stop);
  return hipGetLastError();
}

}  // namespace dgn
