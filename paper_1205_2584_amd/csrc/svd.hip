// Mode-n singular vectors of a dense real tensor: the SVD initialisation of
// the factors (Section 4.5; the comparisons of Section 6 start from it).
//
// A^(n) is the R leading left singular vectors of the unfolding Y_(n), that
// is the leading eigenvectors of the mode-n Gram matrix G_n = Y_(n) Y_(n)^T.
//  1. G_n in FP64 on the matrix cores: 128 x 128 lower tiles, the summation over
//     the other modes split across workgroups (the splits of one tile set stay
//     on one XCD so its L2 serves the shared row blocks), the partial tiles
//     summed in a fixed order, so the result is deterministic.
//  2. Subspace iteration on G_n + sigma_n I, which has the eigenvectors of G_n;
//     sigma_n = 1e-7 trace(G_n) bounds the condition number of every iterate
//     by about 1e7, also for a G_n of low rank.  Each iteration is
//     Z = (G_n + sigma_n I) Q followed by Q = orth(Z), from the caller's random
//     start block.  orth is the shifted Cholesky QR of Fukaya, Kannan,
//     Nakatsukasa, Yamamoto and Yanagisawa (SIAM J. Sci. Comput. 2020), a
//     Cholesky QR of Z^T Z + s I with s = 11 (m b + b (b + 1)) u ||Z||_F^2,
//     followed by two plain Cholesky QR passes.
//  3. Rayleigh-Ritz: H = Q^T (G_n + sigma_n I) Q, its eigenpairs by cyclic
//     two-sided Jacobi rotations (round-robin ordering, b/2 disjoint rotations
//     at a time), A^(n) = Q V for the R largest Ritz values in decreasing order,
//     each column flipped so that its largest-magnitude entry (the first one on
//     ties) is positive.  Singular values are sqrt(theta_r - sigma_n).
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GT = 128;   // Gram tile edge
constexpr int GK = 32;    // summation chunk of a Gram tile
constexpr int GSK = 144;  // stride of the [k][row] LDS layout (rows contiguous)
constexpr int GSR = 36;   // stride of the [row][k] LDS layout (k contiguous)
constexpr int GOP = GK * GSK;  // doubles per staged operand (= GT * GSR)

__device__ __forceinline__ void tri_index(long long id, int& ti, int& tj) {
  ti = (int)((sqrt(8.0 * id + 1.0) - 1.0) / 2.0);
  while ((long long)(ti + 1) * (ti + 2) / 2 <= id) ++ti;
  while ((long long)ti * (ti + 1) / 2 > id) --ti;
  tj = (int)(id - (long long)ti * (ti + 1) / 2);
}

// Barrier that also orders global-memory writes of the workgroup before the
// reads after it (vmcnt(0) and lgkmcnt(0), then the barrier).
__device__ __forceinline__ void sync_block_mem() {
  __builtin_amdgcn_s_waitcnt(0x0070);
  __threadfence_block();
  __syncthreads();
}

// One chunk of GK summation indices on a 128 x 128 tile: wave w owns the
// 64 x 64 quadrant (rows 64 (w / 2), columns 64 (w % 2)) as 4 x 4 blocks of
// v_mfma_f64_16x16x4f64 (lane l: A[l % 16][l / 16], B[l / 16][l % 16], result
// rows l / 16 + 4v, column l % 16).  KR: operands stored [k][row] (stride GSK),
// else [row][k] (stride GSR).  Both strides keep the 64 lanes of an operand read
// on distinct bank pairs within its two LDS cycles.
template <bool KR>
__device__ __forceinline__ void mma_chunk128(const double* Ti, const double* Tj, v4d acc[4][4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rw = 64 * (w >> 1), cw = 64 * (w & 1);
#pragma unroll 2
  for (int k = 0; k < GK; k += 4) {
    const int kk = k + (lane >> 4);
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = rw + 16 * q + (lane & 15), col = cw + 16 * q + (lane & 15);
      a[q] = KR ? Ti[kk * GSK + row] : Ti[row * GSR + kk];
      b[q] = KR ? Tj[kk * GSK + col] : Tj[col * GSR + kk];
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
  }
}

// Partial Gram tiles.  Logical block L = tile + ntile * split; the hardware
// block b runs L = (b % 8) * (gridDim.x / 8) + b / 8, so the consecutive
// logical blocks that share a split (and its row blocks of Y) sit on one XCD.
// part[(split * ntile + tile) * GT^2 + c + GT r] = sum over the split's chunks
// of Y(., GT ti + r, .) Y(., GT tj + c, .).  Diagonal tiles stage one operand.
template <typename T, bool KR, bool CX>
__device__ __forceinline__ void gram_tile(const T* __restrict__ Y, const GramPlan& g, double* __restrict__ part,
                                          int tile, long long split, double* lds) {
  int ti, tj;
  tri_index(tile, ti, tj);
  const bool diag = ti == tj;
  double* Ti = lds;
  double* Tj = diag ? lds : lds + GOP;
  const long long c_begin = split * g.cps;
  const long long c_end = c_begin + g.cps < g.nchunk ? c_begin + g.cps : g.nchunk;
  const long long cpq = (g.P + GK - 1) / GK;  // chunks per q when P > 1
  constexpr int NS = GK * GT / 256;
  T vi[NS], vj[NS];  // widened to FP64 when staged
  // element s of a thread: KR: row r0, k index k0 + 2s; else: k index kc0,
  // row r0 + 8s (256 threads cover 2 k rows x 128 rows, or 32 k x 8 rows)
  const int r0 = KR ? (threadIdx.x & (GT - 1)) : (threadIdx.x >> 5);
  const int k0 = KR ? (threadIdx.x >> 7) : (threadIdx.x & (GK - 1));
  auto load = [&](long long c) {
    if (KR) {  // P == 1: the rows of a chunk are contiguous
      const long long q0 = c * GK + k0;
      const int i = ti * GT + r0, j = tj * GT + r0;
      const T* yi = Y + i + (long long)g.I * q0;
      const T* yj = Y + j + (long long)g.I * q0;
      const long long step = 2LL * g.I;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const bool okq = q0 + 2 * s < g.Q;
        vi[s] = (okq && i < g.I) ? yi[s * step] : T(0);
        if (!diag) vj[s] = (okq && j < g.I) ? yj[s * step] : T(0);
      }
    } else if (!CX) {  // the chunk runs along p, contiguous for each row
      const long long q = c / cpq;
      const long long p0 = (c - q * cpq) * GK;
      const bool okp = p0 + k0 < g.P;
      const int i = ti * GT + r0, j = tj * GT + r0;
      const T* yi = Y + (p0 + k0 + g.P * ((long long)g.I * q + i));
      const T* yj = Y + (p0 + k0 + g.P * ((long long)g.I * q + j));
      const long long step = 8LL * g.P;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        vi[s] = (okp && i + 8 * s < g.I) ? yi[s * step] : T(0);
        if (!diag) vj[s] = (okp && j + 8 * s < g.I) ? yj[s * step] : T(0);
      }
    } else {  // complex, interleaved (re, im): row 2 i + c is part c of complex row i
      const long long q = c / cpq;
      const long long p0 = (c - q * cpq) * GK;
      const bool okp = p0 + k0 < g.P;
      const long long Ic = g.I >> 1;
      const T* yq = Y + 2 * (p0 + k0 + g.P * Ic * q);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int ri = ti * GT + r0 + 8 * s, rj = tj * GT + r0 + 8 * s;
        vi[s] = (okp && ri < g.I) ? yq[(ri & 1) + 2 * g.P * (long long)(ri >> 1)] : T(0);
        if (!diag) vj[s] = (okp && rj < g.I) ? yq[(rj & 1) + 2 * g.P * (long long)(rj >> 1)] : T(0);
      }
    }
  };
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  if (c_begin < c_end) load(c_begin);
  for (long long c = c_begin; c < c_end; ++c) {
    sync_block();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int idx = KR ? (k0 + 2 * s) * GSK + r0 : (r0 + 8 * s) * GSR + k0;
      Ti[idx] = to_f64(vi[s]);
      if (!diag) Tj[idx] = to_f64(vj[s]);
    }
    sync_block();
    if (c + 1 < c_end) load(c + 1);
    mma_chunk128<KR>(Ti, Tj, acc);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rw = 64 * (w >> 1), cw = 64 * (w & 1);
  double* out = part + (split * g.ntile + tile) * (GT * GT);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rw + 16 * rb + (lane >> 4) + 4 * v, c = cw + 16 * cb + (lane & 15);
        out[c + GT * r] = acc[rb][cb][v];
      }
}

template <typename T, bool KR, bool CX = false>
__global__ __launch_bounds__(256, 2) void k_mode_gram(const T* __restrict__ Y, GramPlan g, double* __restrict__ part) {
  __shared__ double lds[2 * GOP];
  const long long per_xcd = gridDim.x / 8;
  const long long L = (long long)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (L >= (long long)g.ntile * g.S) return;
  gram_tile<T, KR, CX>(Y, g, part, (int)(L % g.ntile), L / g.ntile, lds);
}

// The Hermitian G = Y_(n) Y_(n)^H from the real Gram G' of the interleaved rows
// (row 2 i + c = part c of row i): G_re = G'[2i][2j] + G'[2i+1][2j+1],
// G_im = G'[2i+1][2j] - G'[2i][2j+1].  E (leading dimension lde) receives the
// real symmetric embedding [[G_re, -G_im], [G_im, G_re]] (2I x 2I), Gc (when
// not NULL, leading dimension I) the interleaved complex G.
__global__ __launch_bounds__(256) void k_hermitian(const double* __restrict__ Gp, long long ldg, int I,
                                                   double* __restrict__ E, long long lde,
                                                   double* __restrict__ Gc) {
  const long long total = (long long)I * I;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int i = (int)(e % I), j = (int)(e / I);
    const double gre = Gp[2 * i + ldg * (2 * j)] + Gp[2 * i + 1 + ldg * (2 * j + 1)];
    const double gim = Gp[2 * i + 1 + ldg * (2 * j)] - Gp[2 * i + ldg * (2 * j + 1)];
    if (E) {
      E[i + lde * j] = gre;
      E[i + lde * (I + j)] = -gim;
      E[I + i + lde * j] = gim;
      E[I + i + lde * (I + j)] = gre;
    }
    if (Gc) {
      Gc[2 * (i + (long long)I * j)] = gre;
      Gc[2 * (i + (long long)I * j) + 1] = gim;
    }
  }
}

// G[gr + ld gc] = G[gc + ld gr] = sum over splits (in order) of the partial
// tiles, for gr >= gc, gr < lim.  GT^2 / 256 blocks per lower tile, one
// element per thread.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int S, int ntile,
                                                     double* __restrict__ G, long long ld, int lim) {
  constexpr int per_tile = GT * GT / 256;
  const int tile = blockIdx.x / per_tile;
  const int e = (blockIdx.x % per_tile) * 256 + threadIdx.x;
  int ti, tj;
  tri_index(tile, ti, tj);
  const int gr = ti * GT + e / GT, gc = tj * GT + e % GT;
  if (gr < gc || gr >= lim) return;
  double v = 0.0;
  for (int sp = 0; sp < S; ++sp) v += part[((long long)sp * ntile + tile) * (GT * GT) + e];
  G[gr + ld * gc] = v;
  G[gc + ld * gr] = v;
}

// sigma[n] = 1e-7 * trace(G_n); one block per mode.
__global__ __launch_bounds__(256) void k_svd_shift(SvdModes m, double* sigma) {
  __shared__ double red[16];
  const int n = blockIdx.x;
  double t = 0.0;
  for (int i = threadIdx.x; i < m.I[n]; i += 256) t += m.G[n][i + (long long)m.Ip[n] * i];
  t = block_sum(t, red);
  if (threadIdx.x == 0) sigma[n] = 1e-7 * t;
}

// Z_n = Omega_n (I_n x b, column-major, modes stacked) padded to Ip x bp with
// zeros; Q_n = 0 (its padding stays zero for good).
__global__ __launch_bounds__(256) void k_svd_load(SvdModes m, const double* __restrict__ omega) {
  const int n = blockIdx.y;
  const int I = m.I[n], Ip = m.Ip[n];
  long long off = 0;
  for (int k = 0; k < n; ++k) off += (long long)m.I[k] * m.b;
  const long long total = (long long)Ip * m.bp;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int i = (int)(e % Ip), c = (int)(e / Ip);
    m.Z[n][e] = (i < I && c < m.b) ? omega[off + i + (long long)I * c] : 0.0;
    m.Q[n][e] = 0.0;
  }
}

// Complex tensors: Z_n = the real embedding [[W_re, -W_im], [W_im, W_re]] of the
// complex start block W (I_c x b_c, interleaved, modes stacked) in the 2 I_c x
// 2 b_c leading part of the Ip x bp block, zeros elsewhere; Q_n = 0.
__global__ __launch_bounds__(256) void k_svd_load_c(SvdModes m, const double* __restrict__ omega) {
  const int n = blockIdx.y;
  const int Ip = m.Ip[n], Ic = m.I[n] / 2, bc = m.b / 2;
  long long off = 0;
  for (int k = 0; k < n; ++k) off += (long long)(m.I[k] / 2) * bc;
  const long long total = (long long)Ip * m.bp;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int i = (int)(e % Ip), c = (int)(e / Ip);
    double v = 0.0;
    if (i < 2 * Ic && c < 2 * bc) {
      const int ii = i % Ic, cc = c % bc, bi = i / Ic, bc2 = c / bc;
      const double* w = omega + 2 * (off + ii + (long long)Ic * cc);
      v = bi == bc2 ? w[0] : (bi == 1 ? w[1] : -w[1]);
    }
    m.Z[n][e] = v;
    m.Q[n][e] = 0.0;
  }
}

// Complex tensors: the real Ritz vectors of the embedding come in pairs (both
// for one complex singular value); column 2r = [a; b] gives u_r = a + i b,
// scaled by the unit factor that makes its largest-magnitude entry (the first
// on ties) real and positive.  One block per mode, wave w takes r = w, w + 4, ...
__global__ __launch_bounds__(256) void k_svd_complexify(SvdModes m, int R, CxFactors out,
                                                        const double* __restrict__ svr, double* sv) {
  const int n = blockIdx.x, Ic = m.I[n] / 2, I2 = m.I[n];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* V = m.A[n];
  double* A = out.A[n];
  for (int r = w; r < R; r += 4) {
    const double* v = V + (long long)I2 * (2 * r);
    double best = -1.0, bre = 0.0, bim = 0.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < Ic; i += 64) {
      const double re = v[i], im = v[Ic + i];
      const double a = sqrt(re * re + im * im);
      if (a > best) {
        best = a;
        bre = re;
        bim = im;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64), ore = __shfl_xor(bre, o, 64), oim = __shfl_xor(bim, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bre = ore;
        bim = oim;
        bi = oi;
      }
    }
    // phase = conj(u_k) / |u_k|
    const double pr = best > 0.0 ? bre / best : 1.0, pi = best > 0.0 ? -bim / best : 0.0;
    for (int i = lane; i < Ic; i += 64) {
      const double re = v[i], im = v[Ic + i];
      A[2 * (i + (long long)Ic * r)] = re * pr - im * pi;
      A[2 * (i + (long long)Ic * r) + 1] = re * pi + im * pr;
    }
    if (sv && lane == 0) sv[n * R + r] = svr[n * 2 * R + 2 * r];
  }
}

// Z_n = (G_n + sigma_n I) Q_n for every mode: blocks of 64 rows x 16 columns,
// wave w owns rows 16w..16w+15; operands read from L2 (G_n, Q_n stay resident).
__global__ __launch_bounds__(256) void k_gq(SvdModes m, const double* __restrict__ sigma) {
  int n = 0;
  while (n + 1 < m.N && (int)blockIdx.x >= m.blk0[n + 1]) ++n;
  const int Ip = m.Ip[n], rt_count = Ip / 64;
  const int local = blockIdx.x - m.blk0[n];
  const int rt = local % rt_count, cb = local / rt_count;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* G = m.G[n];
  const double* Q = m.Q[n];
  const int row_a = rt * 64 + 16 * w + (lane & 15);
  const int col = cb * 16 + (lane & 15);
  const double* ap = G + row_a + (long long)(lane >> 4) * Ip;
  const double* bp = Q + (lane >> 4) + (long long)col * Ip;
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int k = 0; k < Ip; k += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[(long long)k * Ip], bp[k], acc, 0, 0, 0);
  const double sg = sigma[n];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const long long idx = (rt * 64 + 16 * w + (lane >> 4) + 4 * v) + (long long)col * Ip;
    m.Z[n][idx] = acc[v] + sg * Q[idx];
  }
}

// W[0..b)[0..b) (lower blocks of 16) = X^T Y over the first I rows of the
// Ip x bp column-major X, Y, staged through LDS in chunks of CH rows (the next
// chunk in flight in registers while the current one runs on MFMA).  Waves
// take 16 x 16 blocks (bi, bj) round robin; `lower` limits them to bi >= bj.
template <int BP, int CH>
__device__ void gram_small(const double* X, const double* Y, int I, int Ip, bool lower, double (*W)[BP + 1],
                           double (*Xc)[BP + 1], double (*Yc)[BP + 1]) {
  constexpr int NB = BP / 16;
  constexpr int NPAIR = NB * NB;
  constexpr int NW = 8;
  constexpr int MAXP = (NPAIR + NW - 1) / NW;
  constexpr int NE = CH * BP / 512;  // staged elements per thread
  static_assert(CH * BP % 512 == 0 && 64 % CH == 0, "chunk shape");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool two = Y != X;
  // element s of a thread: row kc of the chunk, column c0 + (512 / CH) s
  const int kc = threadIdx.x % CH, c0 = threadIdx.x / CH;
  double px[NE], py[NE];
  auto load = [&](int r0) {  // r0 + CH <= Ip: r0 < I <= Ip, both multiples of CH | 64 | Ip
#pragma unroll
    for (int s = 0; s < NE; ++s) {
      const long long idx = (r0 + kc) + (long long)(c0 + (512 / CH) * s) * Ip;
      px[s] = X[idx];
      if (two) py[s] = Y[idx];
    }
  };
  v4d acc[MAXP];
#pragma unroll
  for (int p = 0; p < MAXP; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
  if (I > 0) load(0);
  for (int r0 = 0; r0 < I; r0 += CH) {
    sync_block();
#pragma unroll
    for (int s = 0; s < NE; ++s) {
      Xc[kc][c0 + (512 / CH) * s] = px[s];
      if (two) Yc[kc][c0 + (512 / CH) * s] = py[s];
    }
    sync_block();
    if (r0 + CH < I) load(r0 + CH);
    const double (*Yv)[BP + 1] = two ? Yc : Xc;
#pragma unroll
    for (int p = 0; p < MAXP; ++p) {
      const int pr = w + NW * p;
      if (pr >= NPAIR) break;
      const int bi = pr / NB, bj = pr % NB;
      if (lower && bi < bj) continue;
#pragma unroll
      for (int k = 0; k < CH; k += 4) {
        const double a = Xc[k + (lane >> 4)][16 * bi + (lane & 15)];
        const double bb = Yv[k + (lane >> 4)][16 * bj + (lane & 15)];
        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[p], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < MAXP; ++p) {
    const int pr = w + NW * p;
    if (pr >= NPAIR) break;
    const int bi = pr / NB, bj = pr % NB;
    if (lower && bi < bj) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) W[16 * bi + (lane >> 4) + 4 * v][16 * bj + (lane & 15)] = acc[p][v];
  }
  sync_block();
}

// One workgroup (512 threads) per mode: Q_n = orth(Z_n) over the first b
// columns by shifted Cholesky QR and two Cholesky QR passes.  Each pass forms
// W = X^T X, factors W (+ s I in the first pass) = L L^T in LDS and replaces
// every row x of X by the solution of L y^T = x^T.  A non-positive pivot sets
// *bad and leaves Q_n as it is.
template <int BP>
__global__ __launch_bounds__(512) void k_orth(SvdModes m, int* bad) {
  __shared__ double W[BP][BP + 1];
  __shared__ double Xc[64][BP + 1];
  __shared__ double Dinv[BP];
  __shared__ int fail;
  const int n = blockIdx.x;
  const int I = m.I[n], Ip = m.Ip[n], b = m.b;
  const double* Z = m.Z[n];
  double* Q = m.Q[n];
  if (threadIdx.x == 0) fail = 0;
  for (int pass = 0; pass < 3; ++pass) {
    const double* src = pass == 0 ? Z : Q;
    gram_small<BP, 64>(src, src, I, Ip, true, W, Xc, Xc);
    if (pass == 0) {
      double tr = 0.0;
      for (int j = 0; j < b; ++j) tr += W[j][j];
      sync_block();
      const double s = 11.0 * ((double)I * b + (double)b * (b + 1)) * 0x1p-53 * tr;
      if ((int)threadIdx.x < b) W[threadIdx.x][threadIdx.x] += s;
      sync_block();
    }
    // unscaled right-looking Cholesky of the lower triangle: after step j,
    // W[i][k] (k > j) holds the Schur complement, column j the unscaled column.
    for (int j = 0; j < b; ++j) {
      const double d = W[j][j];
      if (!(d > 0.0) || !isfinite(d)) {
        if (threadIdx.x == 0) fail = 1;
        break;
      }
      const double dinv = 1.0 / d;
      for (int i = j + 1 + (int)(threadIdx.x >> 4); i < b; i += 32)
        for (int k = j + 1 + (int)(threadIdx.x & 15); k <= i; k += 16) W[i][k] -= W[i][j] * W[k][j] * dinv;
      sync_block();
    }
    sync_block();
    if (fail) break;
    // Dinv = 1 / diag(L), zero on the padding columns [b, BP), whose rows of W
    // are zero (zero columns of X): the substitution below then leaves them zero
    if ((int)threadIdx.x < BP) Dinv[threadIdx.x] = (int)threadIdx.x < b ? 1.0 / sqrt(W[threadIdx.x][threadIdx.x]) : 0.0;
    sync_block();
    // L[c][k] = W[c][k] / sqrt(W[k][k]) for k < c
    for (int c = 1 + (int)(threadIdx.x >> 4); c < b; c += 32)
      for (int k = threadIdx.x & 15; k < c; k += 16) W[c][k] *= Dinv[k];
    sync_block();
    for (int i = threadIdx.x; i < I; i += 512) {
      // keeps the loads of L inside the loop (hoisted, they would take BP^2 / 2 registers)
      __asm__ volatile("" ::: "memory");
      // all BP columns, unguarded: padding columns are zero in and out
      double x[BP];
#pragma unroll
      for (int c = 0; c < BP; ++c) x[c] = src[i + (long long)c * Ip];
#pragma unroll
      for (int c = 0; c < BP; ++c) {
        double a = x[c];
#pragma unroll
        for (int k = 0; k < c; ++k) a -= W[c][k] * x[k];
        x[c] = a * Dinv[c];
      }
#pragma unroll
      for (int c = 0; c < BP; ++c) Q[i + (long long)c * Ip] = x[c];
    }
    sync_block_mem();
  }
  if (threadIdx.x == 0 && fail) atomicOr(bad, 1);
}

// One workgroup (512 threads) per mode: Rayleigh-Ritz on span(Q_n) with
// Z_n = (G_n + sigma_n I) Q_n, Jacobi eigensolver, Ritz vectors of the R
// largest Ritz values into A_n (I_n x R, leading dimension I_n) and the
// singular values into sv[n R + r] (when sv != NULL).
template <int BP>
__global__ __launch_bounds__(512) void k_rayleigh_ritz(SvdModes m, const double* __restrict__ sigma, double* sv) {
  __shared__ double H[BP][BP + 1];
  __shared__ double V[BP][BP + 1];
  __shared__ double Qc[32][BP + 1];
  __shared__ double Zc[32][BP + 1];
  __shared__ double rc[BP / 2], rs[BP / 2];
  __shared__ int rp[BP / 2], rq[BP / 2];
  __shared__ int rotated;
  __shared__ int perm[BP];
  __shared__ double lam[BP];
  const int n = blockIdx.x;
  const int I = m.I[n], Ip = m.Ip[n], b = m.b, R = m.R;
  const double* Q = m.Q[n];
  gram_small<BP, 32>(Q, m.Z[n], I, Ip, false, H, Qc, Zc);
  const double sg = sigma[n];
  // symmetrise, remove the shift, V = identity
  for (int e = threadIdx.x; e < b * b; e += 512) {
    const int i = e / b, j = e % b;
    if (i < j) {
      const double h = 0.5 * (H[i][j] + H[j][i]);
      H[i][j] = h;
      H[j][i] = h;
    } else if (i == j) {
      H[i][i] -= sg;
    }
  }
  sync_block();
  // V = identity on [0, b), zero elsewhere (the padding rows stay zero)
  for (int e = threadIdx.x; e < BP * BP; e += 512) V[e / BP][e % BP] = (e / BP == e % BP && e / BP < b) ? 1.0 : 0.0;
  sync_block();
  const int bj = b + (b & 1), np = bj / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    sync_block();
    for (int step = 0; step < bj - 1; ++step) {
      if ((int)threadIdx.x < np) {
        const int k = threadIdx.x;
        // round-robin pairing: position 0 fixed, positions 1..bj-1 rotate
        auto at = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + step) % (bj - 1); };
        int p = at(k), q = at(bj - 1 - k);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        bool act = false;
        if (q < b) {
          const double hpq = H[p][q], hpp = H[p][p], hqq = H[q][q];
          if (fabs(hpq) > 1e-300 && fabs(hpq) > 1e-15 * sqrt(fabs(hpp * hqq))) {
            const double th = (hqq - hpp) / (2.0 * hpq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            act = true;
          }
        }
        rc[k] = c;
        rs[k] = s;
        rp[k] = act ? p : -1;
        rq[k] = q;
        if (act) rotated = 1;
      }
      sync_block();
      // rows p, q of H <- J^T H
      for (int e = threadIdx.x; e < np * b; e += 512) {
        const int k = e / b, j = e % b;
        const int p = rp[k];
        if (p < 0) continue;
        const int q = rq[k];
        const double c = rc[k], s = rs[k];
        const double hp = H[p][j], hq = H[q][j];
        H[p][j] = c * hp - s * hq;
        H[q][j] = s * hp + c * hq;
      }
      sync_block();
      // columns p, q of H <- H J and of V <- V J
      for (int e = threadIdx.x; e < np * b; e += 512) {
        const int k = e / b, i = e % b;
        const int p = rp[k];
        if (p < 0) continue;
        const int q = rq[k];
        const double c = rc[k], s = rs[k];
        const double hp = H[i][p], hq = H[i][q];
        H[i][p] = c * hp - s * hq;
        H[i][q] = s * hp + c * hq;
        const double vp = V[i][p], vq = V[i][q];
        V[i][p] = c * vp - s * vq;
        V[i][q] = s * vp + c * vq;
      }
      sync_block();
    }
    if (!rotated) break;
    sync_block();
  }
  // order: decreasing Ritz value, lower index first on ties
  if ((int)threadIdx.x < b) {
    const int j = threadIdx.x;
    const double lj = H[j][j];
    int rank = 0;
    for (int k = 0; k < b; ++k) {
      const double lk = H[k][k];
      rank += (lk > lj) || (lk == lj && k < j);
    }
    perm[rank] = j;
    lam[rank] = lj;
  }
  sync_block();
  double* A = m.A[n];
  for (int i = threadIdx.x; i < I; i += 512) {
    __asm__ volatile("" ::: "memory");
    double q[BP];  // padding columns of Q are zero, as are the padding rows of V
#pragma unroll
    for (int k = 0; k < BP; ++k) q[k] = Q[i + (long long)k * Ip];
    for (int r = 0; r < R; ++r) {
      const int j = perm[r];
      double u = 0.0;
#pragma unroll
      for (int k = 0; k < BP; ++k) u += q[k] * V[k][j];
      A[i + (long long)I * r] = u;
    }
  }
  sync_block_mem();
  // sign of each column: largest |entry| positive (first index on ties)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r = w; r < R; r += 8) {
    double best = -1.0, bval = 0.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < I; i += 64) {
      const double v = A[i + (long long)I * r];
      if (fabs(v) > best) {
        best = fabs(v);
        bval = v;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64), ov = __shfl_xor(bval, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bval = ov;
        bi = oi;
      }
    }
    if (bval < 0.0)
      for (int i = lane; i < I; i += 64) A[i + (long long)I * r] = -A[i + (long long)I * r];
  }
  if (sv && (int)threadIdx.x < R) {
    const double l = lam[threadIdx.x];
    sv[n * R + threadIdx.x] = l > 0.0 ? sqrt(l) : 0.0;
  }
}

template <int BP>
hipError_t launch_orth_rr(const SvdModes& m, bool rr, const double* sigma, double* sv, int* bad, hipStream_t st) {
  if (rr)
    hipLaunchKernelGGL(k_rayleigh_ritz<BP>, dim3(m.N), dim3(512), 0, st, m, sigma, sv);
  else
    hipLaunchKernelGGL(k_orth<BP>, dim3(m.N), dim3(512), 0, st, m, bad);
  return hipGetLastError();
}

hipError_t orth_or_rr(const SvdModes& m, bool rr, const double* sigma, double* sv, int* bad, hipStream_t st) {
  switch (m.bp) {
    case 16: return launch_orth_rr<16>(m, rr, sigma, sv, bad, st);
    case 32: return launch_orth_rr<32>(m, rr, sigma, sv, bad, st);
    case 48: return launch_orth_rr<48>(m, rr, sigma, sv, bad, st);
    case 64: return launch_orth_rr<64>(m, rr, sigma, sv, bad, st);
    case 80: return launch_orth_rr<80>(m, rr, sigma, sv, bad, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

GramPlan plan_gram(const Shape& s, int n) {
  GramPlan g{};
  g.P = 1;
  g.Q = 1;
  for (int k = 0; k < n; ++k) g.P *= s.I[k];
  for (int k = n + 1; k < s.N; ++k) g.Q *= s.I[k];
  g.I = s.I[n];
  const int nt = (g.I + GT - 1) / GT;
  g.ntile = nt * (nt + 1) / 2;
  g.nchunk = g.P == 1 ? (g.Q + GK - 1) / GK : g.Q * ((g.P + GK - 1) / GK);
  // at most 512 workgroups, one round at two per CU, when the summation allows
  long long S = 512 / g.ntile;
  if (S > g.nchunk) S = g.nchunk;
  if (S < 1) S = 1;
  g.cps = (g.nchunk + S - 1) / S;
  g.S = (int)((g.nchunk + g.cps - 1) / g.cps);
  return g;
}

size_t gram_part_doubles(const Shape& s) {
  size_t mx = 0;
  for (int n = 0; n < s.N; ++n) {
    const GramPlan g = plan_gram(s, n);
    const size_t d = (size_t)g.S * g.ntile * GT * GT;
    if (d > mx) mx = d;
  }
  return mx;
}

hipError_t launch_mode_gram(const Shape& s, int n, const void* Y, YType yt, double* part, double* G, long long ld,
                            int lim, hipStream_t st) {
  const GramPlan g = plan_gram(s, n);
  const long long blocks = (long long)g.ntile * g.S;
  const unsigned grid = (unsigned)((blocks + 7) / 8 * 8);
  const bool kr = g.P == 1;  // mode 1: rows of a chunk contiguous in memory
  switch (yt) {
    case YType::F64:
      if (kr) hipLaunchKernelGGL((k_mode_gram<double, true>), dim3(grid), dim3(256), 0, st, (const double*)Y, g, part);
      else hipLaunchKernelGGL((k_mode_gram<double, false>), dim3(grid), dim3(256), 0, st, (const double*)Y, g, part);
      break;
    case YType::F32:
      if (kr) hipLaunchKernelGGL((k_mode_gram<float, true>), dim3(grid), dim3(256), 0, st, (const float*)Y, g, part);
      else hipLaunchKernelGGL((k_mode_gram<float, false>), dim3(grid), dim3(256), 0, st, (const float*)Y, g, part);
      break;
    case YType::BF16:
      if (kr) hipLaunchKernelGGL((k_mode_gram<__bf16, true>), dim3(grid), dim3(256), 0, st, (const __bf16*)Y, g, part);
      else hipLaunchKernelGGL((k_mode_gram<__bf16, false>), dim3(grid), dim3(256), 0, st, (const __bf16*)Y, g, part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3(g.ntile * (GT * GT / 256)), dim3(256), 0, st, part, g.S, g.ntile, G, ld,
                     lim);
  return hipGetLastError();
}

namespace {

// Shift, start block, orthonormalisation, iterations and Rayleigh-Ritz on the
// Grams already in m.G (real, or the embeddings of complex ones).
hipError_t svd_iterate(SvdModes m, bool cplx, const double* omega, int iters, double* sigma, double* sv, int* bad,
                       hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(k_svd_shift, dim3(m.N), dim3(256), 0, st, m, sigma);
  if (cplx)
    hipLaunchKernelGGL(k_svd_load_c, dim3(64, m.N), dim3(256), 0, st, m, omega);
  else
    hipLaunchKernelGGL(k_svd_load, dim3(64, m.N), dim3(256), 0, st, m, omega);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = orth_or_rr(m, false, sigma, sv, bad, st)) != hipSuccess) return e;
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_gq, dim3(m.blk0[m.N]), dim3(256), 0, st, m, sigma);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = orth_or_rr(m, false, sigma, sv, bad, st)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gq, dim3(m.blk0[m.N]), dim3(256), 0, st, m, sigma);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return orth_or_rr(m, true, sigma, sv, bad, st);
}

}  // namespace

hipError_t launch_svd_init(const Shape& s, const void* Y, YType yt, SvdModes m, const double* omega, int iters,
                           double* part, double* sigma, double* sv, int* bad, hipStream_t st) {
  hipError_t e;
  for (int n = 0; n < s.N; ++n)
    if ((e = launch_mode_gram(s, n, Y, yt, part, m.G[n], m.Ip[n], m.Ip[n], st)) != hipSuccess) return e;
  return svd_iterate(m, false, omega, iters, sigma, sv, bad, st);
}

GramPlan plan_gram_c(const Shape& s, int n) {
  GramPlan g = plan_gram(s, n);  // P, Q, chunks in complex elements
  g.I = 2 * s.I[n];              // rows: (re, im) parts of each complex row
  const int nt = (g.I + GT - 1) / GT;
  g.ntile = nt * (nt + 1) / 2;
  long long S = 512 / g.ntile;
  if (S > g.nchunk) S = g.nchunk;
  if (S < 1) S = 1;
  g.cps = (g.nchunk + S - 1) / S;
  g.S = (int)((g.nchunk + g.cps - 1) / g.cps);
  return g;
}

size_t gram_part_doubles_c(const Shape& s) {
  size_t mx = 0;
  for (int n = 0; n < s.N; ++n) {
    const GramPlan g = plan_gram_c(s, n);
    const size_t d = (size_t)g.S * g.ntile * GT * GT;
    if (d > mx) mx = d;
  }
  return mx;
}

hipError_t launch_mode_gram_c(const Shape& s, int n, const void* Y, YType yt, double* part, double* Gp,
                              double* E, long long lde, double* Gc, hipStream_t st) {
  const GramPlan g = plan_gram_c(s, n);
  const long long blocks = (long long)g.ntile * g.S;
  const unsigned grid = (unsigned)((blocks + 7) / 8 * 8);
  // mode 1: the interleaved rows of a chunk are contiguous, the real kernel applies
  const bool kr = g.P == 1;
  switch (yt) {
    case YType::C128:
      if (kr) hipLaunchKernelGGL((k_mode_gram<double, true>), dim3(grid), dim3(256), 0, st, (const double*)Y, g, part);
      else hipLaunchKernelGGL((k_mode_gram<double, false, true>), dim3(grid), dim3(256), 0, st, (const double*)Y, g, part);
      break;
    case YType::C64:
      if (kr) hipLaunchKernelGGL((k_mode_gram<float, true>), dim3(grid), dim3(256), 0, st, (const float*)Y, g, part);
      else hipLaunchKernelGGL((k_mode_gram<float, false, true>), dim3(grid), dim3(256), 0, st, (const float*)Y, g, part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3(g.ntile * (GT * GT / 256)), dim3(256), 0, st, part, g.S, g.ntile, Gp,
                     (long long)g.I, g.I);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hermitian, dim3(256), dim3(256), 0, st, Gp, (long long)g.I, s.I[n], E, lde, Gc);
  return hipGetLastError();
}

hipError_t launch_svd_init_c(const Shape& s, const void* Y, YType yt, SvdModes m, CxFactors out, double* Gp,
                             const double* omega, int iters, double* part, double* sigma, double* svr, double* sv,
                             int* bad, hipStream_t st) {
  hipError_t e;
  for (int n = 0; n < s.N; ++n) {
    // the embedding fills 2 I_n x 2 I_n; its padding to Ip must be zero
    if ((e = hipMemsetAsync(m.G[n], 0, sizeof(double) * m.Ip[n] * m.Ip[n], st)) != hipSuccess) return e;
    if ((e = launch_mode_gram_c(s, n, Y, yt, part, Gp, m.G[n], m.Ip[n], nullptr, st)) != hipSuccess) return e;
  }
  if ((e = svd_iterate(m, true, omega, iters, sigma, svr, bad, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_svd_complexify, dim3(m.N), dim3(256), 0, st, m, m.R / 2, out, svr, sv);
  return hipGetLastError();
}

}  // namespace dgn
