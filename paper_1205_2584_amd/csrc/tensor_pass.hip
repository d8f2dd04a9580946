// One pass over a dense tensor computing the MTTKRP of every mode
// (Section 4.4: Y_(n) times the Khatri-Rao product of the other factors, the
// O(NRJ) step of Algorithm 1), optionally on the residual E = Y - Y_hat formed
// on the fly (residual-corrected gradient).
//
// Y (first index fastest) is viewed as I_1 x I_2 x Q with Q = prod_{k>=3} I_k
// and c_q[r] = prod_{k>=3} A^(k)[i_k(q), r].  For every slab Y_q:
//   Z_q = Y_q A^(2)      -> M_1 += Z_q diag(c_q)
//   W_q = Y_q^T A^(1)    -> M_2 += W_q diag(c_q)
//   t_q[r] = sum_i A^(1)[i,r] Z_q[i,r]  -> the trailing modes' MTTKRP from t.
// Every element of Y is read once; the contraction costs 4 J R flops.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

struct PassArgs {
  const void* Y;
  int I0, I1, N, R;
  long long Q;
  int It[kMaxOrder];   // I_3..I_N (trailing dims), It[k-2] for mode k
  const double* A;     // stacked FP64 factors
  int off[kMaxOrder];  // element offsets (row offset * R) of each mode's block
  int tiles_i, tiles_j, q_per;
  void* m0part;  // [n_qc][tiles_j][R][I0]
  void* m1part;  // [n_qc][tiles_i][R][I1]
  void* tpart;   // [tiles_i*tiles_j][R][Q]
  double* e2part;
};

template <typename TY>
__device__ __forceinline__ float load_cvt(const TY* p, long long i, float*) { return to_f32(p[i]); }
__device__ __forceinline__ double load_cvt(const double* p, long long i, double*) { return p[i]; }

// Generic FMA version: TC = double for FP64 tensors, float otherwise.
template <typename TY, typename TC, bool RESID>
__global__ __launch_bounds__(256) void k_pass_fma(PassArgs a, const int* stop) {
  if (stopped(stop)) return;
  __shared__ TC Ys[64][65];                 // Ys[jj][ii] = Y[i0+ii, j0+jj, q]
  __shared__ TC A0s[64][kMaxRank + 1];      // A^(1) rows of the tile
  __shared__ TC A1s[64][kMaxRank + 1];      // A^(2) rows of the tile
  __shared__ TC A1c[RESID ? 64 : 1][kMaxRank + 1];  // A^(2) diag(c_q), residual only
  __shared__ TC cq[kMaxRank];
  __shared__ double red[16];

  const int t = threadIdx.x, lane = t & 63, rg = t >> 6;
  const int R = a.R, I0 = a.I0, I1 = a.I1;
  const int tile = blockIdx.x;
  const int tj = tile % a.tiles_j, ti = tile / a.tiles_j;
  const int i0 = ti * 64, j0 = tj * 64;
  const long long q0 = (long long)blockIdx.y * a.q_per;
  long long q1 = q0 + a.q_per;
  if (q1 > a.Q) q1 = a.Q;
  const TY* Y = static_cast<const TY*>(a.Y);

  for (int e = t; e < 64 * kMaxRank; e += 256) {
    const int ii = e & 63, r = e >> 6;
    const int gi = i0 + ii, gj = j0 + ii;
    A0s[ii][r] = (r < R && gi < I0) ? (TC)a.A[a.off[0] + gi + (long long)r * I0] : (TC)0;
    A1s[ii][r] = (r < R && gj < I1) ? (TC)a.A[a.off[1] + gj + (long long)r * I1] : (TC)0;
  }

  const int KR = (R + 3) / 4;
  TC m0[16], m1[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) { m0[k] = 0; m1[k] = 0; }
  double e2 = 0.0;

  for (long long q = q0; q < q1; ++q) {
    sync_block();
    // stage the 64 x 64 slab tile (coalesced along the first index)
    const long long base = (long long)I0 * I1 * q;
#pragma unroll 4
    for (int e = t; e < 64 * 64; e += 256) {
      const int ii = e & 63, jj = e >> 6;
      const int gi = i0 + ii, gj = j0 + jj;
      TC v = 0;
      if (gi < I0 && gj < I1) v = (TC)to_f64(Y[base + gi + (long long)I0 * gj]);
      Ys[jj][ii] = v;
    }
    if (t < R) {
      double c = 1.0;
      long long qq = q;
      for (int k = 2; k < a.N; ++k) {
        const int Ik = a.It[k - 2];
        const int ik = (int)(qq % Ik);
        qq /= Ik;
        c *= a.A[a.off[k] + ik + (long long)t * Ik];
      }
      cq[t] = (TC)c;
    }
    sync_block();
    if (RESID) {
      for (int e = t; e < 64 * kMaxRank; e += 256) {
        const int jj = e & 63, r = e >> 6;
        A1c[jj][r] = A1s[jj][r] * (r < R ? cq[r] : (TC)0);
      }
      sync_block();
      for (int e = t; e < 64 * 64; e += 256) {
        const int ii = e & 63, jj = e >> 6;
        TC yh = 0;
        for (int r = 0; r < R; ++r) yh += A0s[ii][r] * A1c[jj][r];
        const TC ev = Ys[jj][ii] - yh;  // zero outside the tensor (both terms vanish)
        e2 += (double)ev * (double)ev;
        Ys[jj][ii] = ev;
      }
      sync_block();
    }
    TC zp[16], wp[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) { zp[k] = 0; wp[k] = 0; }
    for (int jj = 0; jj < 64; ++jj) {
      const TC yv = Ys[jj][lane];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < KR) zp[k] += yv * A1s[jj][rg + 4 * k];
    }
    for (int ii = 0; ii < 64; ++ii) {
      const TC yv = Ys[lane][ii];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < KR) wp[k] += yv * A0s[ii][rg + 4 * k];
    }
    TC* tp = static_cast<TC*>(a.tpart) + (long long)tile * R * a.Q;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k < KR) {
        const int r = rg + 4 * k;
        const TC c = (r < R) ? cq[r] : (TC)0;
        m0[k] += c * zp[k];
        m1[k] += c * wp[k];
        const TC tv = wave_sum(A0s[lane][r] * zp[k]);
        if (lane == 0 && r < R) tp[(long long)r * a.Q + q] = tv;
      }
    }
  }
  // partial MTTKRPs of modes 1 and 2 for this tile and q-chunk
  TC* m0p = static_cast<TC*>(a.m0part) + ((long long)blockIdx.y * a.tiles_j + tj) * R * I0;
  TC* m1p = static_cast<TC*>(a.m1part) + ((long long)blockIdx.y * a.tiles_i + ti) * R * I1;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = rg + 4 * k;
    if (k < KR && r < R) {
      if (i0 + lane < I0) m0p[(long long)r * I0 + i0 + lane] = m0[k];
      if (j0 + lane < I1) m1p[(long long)r * I1 + j0 + lane] = m1[k];
    }
  }
  if (RESID) {
    const double s = block_sum(e2, red);
    if (t == 0) a.e2part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// MFMA versions.  The slab tile (64 x 64, Ys[j][i] in LDS, i contiguous) feeds
//   Z_q = Y_q A^(2):   v_mfma A-operand Y[i][j] (lane: i = 16w + l%16, k = j)
//   W_q = Y_q^T A^(1): v_mfma A-operand Y^T[j][i] (lane: j = 16w + l%16, k = i)
// The factor operands are loop constants held in registers.  The summation
// index of W_q is permuted inside each 16-wide k block so that every lane
// reads four (FP32) or eight (BF16) consecutive i with one LDS vector load;
// the factor operand uses the same permutation.  Result layout of both
// 16x16 instructions: D[4 (l/16) + v][l%16].
// Tiles are numbered with the j-tile fastest.  Workgroups are dealt to the
// XCDs in turn, so a run of consecutive workgroups shares one i-tile row and
// each XCD sees the i-neighbours of its tiles; their row segments share the
// 128-byte lines at the tile edges, which then meet in one L2.
// ---------------------------------------------------------------------------

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int kQMax = 16;  // slabs per block of the MFMA kernels (t and c_q staged in LDS)
// Slabs in flight ahead of the computed one (the ring of slab registers): the
// FP32 slab takes about 2k MFMA cycles per wave, the BF16 slab a fraction of
// that, and both must cover the HBM latency (measured: a ring of two 16 KB
// slabs per workgroup streams the tensor at 6.2 TB/s when nothing else runs).
// The compiler waits for the whole ring once per revolution, so the ring is
// deep enough that a revolution covers that latency; ranks above 32 keep the
// shorter ring so that two workgroups still fit on a CU.  kQMax is a multiple
// of every depth.
template <int NB> constexpr int kPrefetchF32 = NB <= 2 ? 4 : 2;
template <int NB> constexpr int kPrefetchBf16 = NB <= 2 ? 8 : 4;
static_assert(kQMax % kPrefetchF32<1> == 0 && kQMax % kPrefetchBf16<1> == 0 && kQMax % kPrefetchF32<4> == 0 &&
                  kQMax % kPrefetchBf16<4> == 0,
              "sub-chunks align with the ring");

__device__ __forceinline__ float fac(const PassArgs& a, int mode, int Im, int i, int r) {
  return (i < Im && r < a.R) ? (float)a.A[a.off[mode] + i + (long long)r * Im] : 0.0f;
}

__device__ __forceinline__ float cq_of(const PassArgs& a, long long q, int r) {
  if (r >= a.R) return 0.0f;
  double c = 1.0;
  long long qq = q;
  for (int k = 2; k < a.N; ++k) {
    const int Ik = a.It[k - 2];
    const int ik = (int)(qq % Ik);
    qq /= Ik;
    c *= a.A[a.off[k] + ik + (long long)r * Ik];
  }
  return (float)c;
}

// c_q of a sub-chunk of kQMax slabs starting at qs: thread t holds the entries
// e = t + 256 k (slab qs + e / 64, rank e % 64).  For order 3 c_q is a row of
// A^(3), read with unconditional loads (clamped indices, masked on use) one
// sub-chunk ahead of its use, so that its wait never drains the slab ring;
// higher orders form the products when the sub-chunk starts.
struct CqFetch {
  double v[4];
};
__device__ __forceinline__ void cq_prefetch(const PassArgs& a, long long qs, CqFetch& f) {
  if (a.N != 3) return;
  const int I3 = a.It[0];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = threadIdx.x + 256 * k, r = e & 63;
    const long long q = qs + (e >> 6);
    const long long qc = q < a.Q ? q : a.Q - 1;
    const int rc = r < a.R ? r : a.R - 1;
    f.v[k] = a.A[a.off[2] + qc + (long long)rc * I3];
  }
}
__device__ __forceinline__ void cq_stage(const PassArgs& a, long long qs, long long q1, const CqFetch& f,
                                         float (*cq_all)[64]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = threadIdx.x + 256 * k, ql = e >> 6, r = e & 63;
    const bool ok = qs + ql < q1 && r < a.R;
    cq_all[ql][r] = ok ? (a.N == 3 ? (float)f.v[k] : cq_of(a, qs + ql, r)) : 0.0f;
  }
}

// Sum over the four 16-lane rows of the wave (lane l gets the sum over the lanes
// l mod 16 + 16 g): one swap of odd and even rows, then of the two halves, in
// the order ((x0 + x1) + (x2 + x3)) for the lanes of row 0.
__device__ __forceinline__ float sum_rows(float x) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  const float y = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(y), __float_as_uint(y), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// t of the slabs [q0, q1) (at most kQMax, staged per wave in LDS) to the tile's partial.
__device__ __forceinline__ void flush_t(const PassArgs& a, float (*tq_s)[kQMax][64], long long q0, long long q1,
                                        int tile) {
  const int t = threadIdx.x, R = a.R;
  sync_block();
  float* tp = static_cast<float*>(a.tpart) + (long long)tile * R * a.Q;
  const int nq = (int)(q1 - q0);
  for (int e = t; e < nq * R; e += 256) {
    const int ql = e % nq, r = e / nq;
    tp[(long long)r * a.Q + q0 + ql] = ((tq_s[0][ql][r] + tq_s[1][ql][r]) + tq_s[2][ql][r]) + tq_s[3][ql][r];
  }
}

// Partial M_1 and M_2 of the block's tile and q-chunk.
template <int NB>
__device__ __forceinline__ void write_m(const PassArgs& a, int ti, int tj, int i0, int j0, const v4f* m0acc,
                                        const v4f* m1acc) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, c16 = lane & 15;
  const int R = a.R, I0 = a.I0, I1 = a.I1;
  float* m0p = static_cast<float*>(a.m0part) + ((long long)blockIdx.y * a.tiles_j + tj) * R * I0;
  float* m1p = static_cast<float*>(a.m1part) + ((long long)blockIdx.y * a.tiles_i + ti) * R * I1;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int r = 16 * nb + c16;
    if (r < R) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = i0 + 16 * w + 4 * g + v, jj = j0 + 16 * w + 4 * g + v;
        if (ii < I0) m0p[(long long)r * I0 + ii] = m0acc[nb][v];
        if (jj < I1) m1p[(long long)r * I1 + jj] = m1acc[nb][v];
      }
    }
  }
}

// VEC: I_1 is a multiple of 4, so every 4-element piece of a slab row is one
// aligned 16-byte load (a separate instantiation keeps the load sequence free of
// branches, which lets the compiler wait for each slab's loads alone).
template <int NB, bool RESID, bool VEC>
__global__ __launch_bounds__(256) void k_pass_f32(PassArgs a, const int* stop) {
  if (stopped(stop)) return;
  constexpr int LDY = 68;
  // Ys[slab parity][j][i]: the slab is written into one buffer while the other
  // may still be read, so one barrier per slab suffices.  The residual form keeps
  // one buffer (and a second barrier) to stay at two workgroups per CU.
  constexpr int NBUF = RESID ? 1 : 2;
  __shared__ __attribute__((aligned(16))) float Ysb[NBUF][64][LDY];
  __shared__ float cq_all[kQMax][64];
  __shared__ float tq_s[4][kQMax][64];  // per-wave partial t, summed in wave order
  __shared__ float A0s[RESID ? 64 : 1][65];
  __shared__ float A1s[RESID ? 64 : 1][65];
  __shared__ double red[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, c16 = lane & 15;
  const int I0 = a.I0, I1 = a.I1;
  const int tile = blockIdx.x, tj = tile % a.tiles_j, ti = tile / a.tiles_j;
  const int i0 = ti * 64, j0 = tj * 64;
  const long long q0 = (long long)blockIdx.y * a.q_per;
  const long long q1 = (q0 + a.q_per < a.Q) ? q0 + a.q_per : a.Q;
  const float* Y = static_cast<const float*>(a.Y);

  float b1[16][NB], b0[16][NB], a0t[NB][4];
#pragma unroll
  for (int ks = 0; ks < 16; ++ks)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      b1[ks][nb] = fac(a, 1, I1, j0 + 4 * ks + g, 16 * nb + c16);
      b0[ks][nb] = fac(a, 0, I0, i0 + 16 * (ks >> 2) + 4 * g + (ks & 3), 16 * nb + c16);
    }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v) a0t[nb][v] = fac(a, 0, I0, i0 + 16 * w + 4 * g + v, 16 * nb + c16);
  if (RESID) {
    for (int e = t; e < 64 * 64; e += 256) {
      const int ii = e & 63, r = e >> 6;
      A0s[ii][r] = fac(a, 0, I0, i0 + ii, r);
      A1s[ii][r] = fac(a, 1, I1, j0 + ii, r);
    }
  }

  v4f m0acc[NB], m1acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { m0acc[nb] = v4f{0, 0, 0, 0}; m1acc[nb] = v4f{0, 0, 0, 0}; }
  double e2 = 0.0;

  // Slab loads run kPrefetchF32<NB> slabs ahead of the slab being computed.  Every
  // load is unconditional (a piece outside the tensor reads the slab's first
  // elements) and the piece is masked when it is stored to LDS: a load under a
  // branch makes the compiler wait for all outstanding loads (vmcnt(0)) before
  // the slab store, which serialised the ring.  pn: elements of the piece inside
  // the tensor (0..4); poff: its offset within the slab.
  long long poff[4];
  int pn[4];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    const int e = t + 256 * s2, jj = e >> 4, ii = (e & 15) * 4;
    const int gi = i0 + ii, gj = j0 + jj;
    const int n = (gj < I1) ? (I0 - gi < 0 ? 0 : (I0 - gi > 4 ? 4 : I0 - gi)) : 0;
    pn[s2] = n;
    poff[s2] = n > 0 ? (long long)gj * I0 + gi : 0;
  }
  v4f pf[kPrefetchF32<NB>][4];
  auto load = [&](long long q, v4f (&dst)[4]) {
    const float* base = Y + (long long)I0 * I1 * q;
    if constexpr (VEC) {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) dst[s2] = *reinterpret_cast<const v4f*>(base + poff[s2]);
    } else {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[s2][k] = base[poff[s2] + (k < pn[s2] ? k : 0)];
    }
  };
  auto masked = [&](const v4f& v, int s2) {
    v4f m;
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = k < pn[s2] ? v[k] : 0.0f;
    return m;
  };

  // the ring is filled and refilled unconditionally (past the chunk's end the
  // last slab is read again and never used), so every load of the loop sits
  // on the straight-line path and each slab waits only for its own loads
#pragma unroll
  for (int d = 0; d < kPrefetchF32<NB>; ++d) load(q0 + d < q1 ? q0 + d : q1 - 1, pf[d]);
  CqFetch cqf;
  cq_prefetch(a, q0, cqf);
  for (long long qb = q0; qb < q1; qb += kPrefetchF32<NB>) {
  if ((qb - q0) % kQMax == 0) {
    // new sub-chunk of at most kQMax slabs: t of the previous one flushed, c_q
    // staged from the prefetched values, the next sub-chunk's c_q fetched
    if (qb > q0) flush_t(a, tq_s, qb - kQMax, qb, tile);
    cq_stage(a, qb, q1, cqf, cq_all);
    cq_prefetch(a, qb + kQMax, cqf);
  }
#pragma unroll
  for (int d = 0; d < kPrefetchF32<NB>; ++d) {
    const long long q = qb + d;
    const bool live = q < q1;  // uniform over the workgroup
    const int ql = (int)((q - q0) % kQMax);
    float (*Ys)[LDY] = Ysb[(q - q0) & (NBUF - 1)];
    if (live) {
      if (NBUF == 1) sync_block();
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int e = t + 256 * s2, jj = e >> 4, ii = (e & 15) * 4;
        *reinterpret_cast<v4f*>(&Ys[jj][ii]) = masked(pf[d][s2], s2);
      }
    }
    load(q + kPrefetchF32<NB> < q1 ? q + kPrefetchF32<NB> : q1 - 1, pf[d]);
    if (!live) continue;
    const float* cq_s = cq_all[ql];
    sync_block();
    if (RESID) {
      constexpr int KS = NB * 4;  // R padded to 16, in steps of 4
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        v4f acc = v4f{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const float av = A0s[16 * w + c16][4 * ks + g];
          const float bv = cq_s[4 * ks + g] * A1s[16 * jb + c16][4 * ks + g];
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ii = 16 * w + 4 * g + v, jj = 16 * jb + c16;
          const float ev = Ys[jj][ii] - acc[v];
          e2 += (double)ev * (double)ev;
          Ys[jj][ii] = ev;
        }
      }
      sync_block();
    }
    v4f zacc[NB], wacc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) { zacc[nb] = v4f{0, 0, 0, 0}; wacc[nb] = v4f{0, 0, 0, 0}; }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const float av = Ys[4 * ks + g][16 * w + c16];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        zacc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b1[ks][nb], zacc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const v4f y4 = *reinterpret_cast<const v4f*>(&Ys[16 * w + c16][16 * kb + 4 * g]);
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          wacc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(y4[s2], b0[4 * kb + s2][nb], wacc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float c = cq_s[16 * nb + c16];
      m0acc[nb] += c * zacc[nb];
      m1acc[nb] += c * wacc[nb];
      const float tv = sum_rows(a0t[nb][0] * zacc[nb][0] + a0t[nb][1] * zacc[nb][1] + a0t[nb][2] * zacc[nb][2] +
                                a0t[nb][3] * zacc[nb][3]);
      if (g == 0) tq_s[w][ql][16 * nb + c16] = tv;
    }
  }
  }
  if (q0 < q1) flush_t(a, tq_s, q0 + ((q1 - q0 - 1) / kQMax) * kQMax, q1, tile);
  write_m<NB>(a, ti, tj, i0, j0, m0acc, m1acc);
  if (RESID) {
    const double s2 = block_sum(e2, red);
    if (t == 0) a.e2part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s2;
  }
}

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// BF16 tensor: 16x16x32 BF16 MFMA with FP32 accumulation.  Factors enter as
// hi + lo BF16 pairs (two instructions), so only the tensor's own rounding
// remains at the BF16 level.
template <int NB, bool VEC>
__global__ __launch_bounds__(256) void k_pass_bf16(PassArgs a, const int* stop) {
  if (stopped(stop)) return;
  constexpr int LDY = 72;
  // Ys[slab parity][j][i]: one barrier per slab (see k_pass_f32)
  __shared__ __attribute__((aligned(16))) __bf16 Ysb[2][64][LDY];
  __shared__ float cq_all[kQMax][64];
  __shared__ float tq_s[4][kQMax][64];  // per-wave partial t, summed in wave order
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, c16 = lane & 15;
  const int I0 = a.I0, I1 = a.I1;
  const int tile = blockIdx.x, tj = tile % a.tiles_j, ti = tile / a.tiles_j;
  const int i0 = ti * 64, j0 = tj * 64;
  const long long q0 = (long long)blockIdx.y * a.q_per;
  const long long q1 = (q0 + a.q_per < a.Q) ? q0 + a.q_per : a.Q;
  const __bf16* Y = static_cast<const __bf16*>(a.Y);

  v8bf b1h[2][NB], b1l[2][NB], b0h[2][NB], b0l[2][NB];
  float a0t[NB][4];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) {
        __bf16 h, l;
        split_bf16(fac(a, 1, I1, j0 + 32 * ks + 8 * g + tt, 16 * nb + c16), h, l);
        b1h[ks][nb][tt] = h;
        b1l[ks][nb][tt] = l;
        split_bf16(fac(a, 0, I0, i0 + 32 * ks + 8 * g + tt, 16 * nb + c16), h, l);
        b0h[ks][nb][tt] = h;
        b0l[ks][nb][tt] = l;
      }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v) a0t[nb][v] = fac(a, 0, I0, i0 + 16 * w + 4 * g + v, 16 * nb + c16);

  v4f m0acc[NB], m1acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { m0acc[nb] = v4f{0, 0, 0, 0}; m1acc[nb] = v4f{0, 0, 0, 0}; }

  typedef unsigned short us4 __attribute__((ext_vector_type(4)));
  // slab loads run kPrefetchBf16<NB> slabs ahead of the slab being computed
  us4 pf[kPrefetchBf16<NB>][4];
  // this thread's four 4-element pieces of a slab: offset within the slab and
  // how many of the 4 elements lie inside the tensor (an out-of-range piece
  // reads the slab's first element; every load is unconditional and the piece
  // is masked only when it is stored to LDS, so that the compiler waits for
  // each slab's own loads and not for the whole ring)
  long long poff[4];
  int pn[4];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    const int e = t + 256 * s2, jj = e >> 4, ii = (e & 15) * 4;
    const int gi = i0 + ii, gj = j0 + jj;
    const int n = (gj < I1) ? (I0 - gi < 0 ? 0 : (I0 - gi > 4 ? 4 : I0 - gi)) : 0;
    pn[s2] = n;
    poff[s2] = n > 0 ? (long long)gj * I0 + gi : 0;
  }
  auto load = [&](long long q, us4 (&dst)[4]) {
    const unsigned short* base = reinterpret_cast<const unsigned short*>(Y) + (long long)I0 * I1 * q;
    if constexpr (VEC) {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) dst[s2] = *reinterpret_cast<const us4*>(base + poff[s2]);
    } else {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[s2][k] = base[poff[s2] + (k < pn[s2] ? k : 0)];
    }
  };
  auto masked = [&](const us4& v, int s2) {
    us4 m;
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = k < pn[s2] ? v[k] : (unsigned short)0;
    return m;
  };
  // the ring is filled and refilled unconditionally (past the chunk's end the
  // last slab is read again and never used), so every load of the loop sits
  // on the straight-line path and each slab waits only for its own loads
#pragma unroll
  for (int d = 0; d < kPrefetchBf16<NB>; ++d) load(q0 + d < q1 ? q0 + d : q1 - 1, pf[d]);
  CqFetch cqf;
  cq_prefetch(a, q0, cqf);
  for (long long qb = q0; qb < q1; qb += kPrefetchBf16<NB>) {
  if ((qb - q0) % kQMax == 0) {
    // new sub-chunk of at most kQMax slabs: t of the previous one flushed, c_q
    // staged from the prefetched values, the next sub-chunk's c_q fetched
    if (qb > q0) flush_t(a, tq_s, qb - kQMax, qb, tile);
    cq_stage(a, qb, q1, cqf, cq_all);
    cq_prefetch(a, qb + kQMax, cqf);
  }
#pragma unroll
  for (int d = 0; d < kPrefetchBf16<NB>; ++d) {
    const long long q = qb + d;
    const bool live = q < q1;  // uniform over the workgroup
    const int ql = (int)((q - q0) % kQMax);
    __bf16 (*Ys)[LDY] = Ysb[(q - q0) & 1];
    if (live) {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int e = t + 256 * s2, jj = e >> 4, ii = (e & 15) * 4;
        *reinterpret_cast<us4*>(&Ys[jj][ii]) = masked(pf[d][s2], s2);
      }
    }
    load(q + kPrefetchBf16<NB> < q1 ? q + kPrefetchBf16<NB> : q1 - 1, pf[d]);
    if (!live) continue;
    const float* cq_s = cq_all[ql];
    sync_block();
    v4f zacc[NB], wacc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) { zacc[nb] = v4f{0, 0, 0, 0}; wacc[nb] = v4f{0, 0, 0, 0}; }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      v8bf av;
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) av[tt] = Ys[32 * ks + 8 * g + tt][16 * w + c16];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        zacc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1h[ks][nb], zacc[nb], 0, 0, 0);
        zacc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1l[ks][nb], zacc[nb], 0, 0, 0);
      }
      const v8bf yv = *reinterpret_cast<const v8bf*>(&Ys[16 * w + c16][32 * ks + 8 * g]);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        wacc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv, b0h[ks][nb], wacc[nb], 0, 0, 0);
        wacc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv, b0l[ks][nb], wacc[nb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float c = cq_s[16 * nb + c16];
      m0acc[nb] += c * zacc[nb];
      m1acc[nb] += c * wacc[nb];
      const float tv = sum_rows(a0t[nb][0] * zacc[nb][0] + a0t[nb][1] * zacc[nb][1] + a0t[nb][2] * zacc[nb][2] +
                                a0t[nb][3] * zacc[nb][3]);
      if (g == 0) tq_s[w][ql][16 * nb + c16] = tv;
    }
  }
  }
  if (q0 < q1) flush_t(a, tq_s, q0 + ((q1 - q0 - 1) / kQMax) * kQMax, q1, tile);
  write_m<NB>(a, ti, tj, i0, j0, m0acc, m1acc);
}

// out[x] = sum_s part[s * len + x], accumulated in FP64.  A block covers 64
// consecutive x; its 16 waves split the slots.
struct SlotSeg {
  const void* part;  // nslots partial arrays of len values each
  int nslots;
  long long len;
  double* out;
};

// The slot sums of one pass in one launch: blocks [0, nb[0]) sum mode 1's
// partials, the next nb[1] mode 2's, the next nb[2] the t vectors, 64 outputs
// per block.  Optional folds: ipart[b] = sum of A_1[x] M_1[x] over the 64
// outputs of mode-1 block b (the <A_1, M_1> of the error formula in pieces);
// and N + 1 blocks after the slots that sum the row-chunk Gram partials of the
// candidate factors into gout (N R^2) and the two per-row scalars into gscal.
struct ReduceArgs {
  SlotSeg seg[3];
  int nb[3];
  const double* A1;
  double* ipart;
  const double* rowpart;
  int N, chunks, stride, R2;
  double* gout;
  double* gscal;
};

template <typename TC>
__global__ __launch_bounds__(1024) void k_reduce_slots(ReduceArgs ra, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double red[16][65];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  int b = blockIdx.x, sg = 0;
  while (sg < 3 && b >= ra.nb[sg]) b -= ra.nb[sg++];
  if (sg == 3) {
    // Gram partials: block b < N sums mode b, block N the two scalars
    const int t = threadIdx.x;
    if (b == ra.N) {
      if (t < 2) {
        double acc = 0.0;
        for (int m = 0; m < ra.N; ++m)
          for (int c = 0; c < ra.chunks; ++c) acc += ra.rowpart[((long long)m * ra.chunks + c) * ra.stride + ra.R2 + t];
        ra.gscal[t] = acc;
      }
      return;
    }
    for (int x = t; x < ra.R2; x += blockDim.x) {
      double acc = 0.0;
      for (int c = 0; c < ra.chunks; ++c) acc += ra.rowpart[((long long)b * ra.chunks + c) * ra.stride + x];
      ra.gout[(long long)b * ra.R2 + x] = acc;
    }
    return;
  }
  const SlotSeg sd = ra.seg[sg];
  const TC* part = static_cast<const TC*>(sd.part);
  const int nslots = sd.nslots;
  const long long len = sd.len;
  const long long x = b * 64LL + lane;
  double s = 0.0;
  if (x < len) {
    int k = g;
    for (; k + 48 < nslots; k += 64) {
      const double a0 = (double)part[(long long)k * len + x];
      const double a1 = (double)part[(long long)(k + 16) * len + x];
      const double a2 = (double)part[(long long)(k + 32) * len + x];
      const double a3 = (double)part[(long long)(k + 48) * len + x];
      s += (a0 + a1) + (a2 + a3);
    }
    for (; k < nslots; k += 16) s += (double)part[(long long)k * len + x];
  }
  red[g][lane] = s;
  sync_block();
  if (g == 0) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) v += red[i][lane];
    if (x < len) sd.out[x] = v;
    if (sg == 0 && ra.ipart) {
      const double p = wave_sum(x < len ? ra.A1[x] * v : 0.0);
      if (lane == 0) ra.ipart[b] = p;
    }
  }
}

// MTTKRP of the trailing modes k >= 3 from t[q, r] (Q x R, FP64):
// M_k[i, r] = sum_{q : i_k(q) = i} t[q, r] prod_{l >= 3, l != k} A^(l)[i_l(q), r].
__global__ void k_modes_from_t(PassArgs a, const double* tq, double* M, const int* stop) {
  if (stopped(stop)) return;
  const int R = a.R;
  long long total = 0;
  for (int k = 2; k < a.N; ++k) total += (long long)a.It[k - 2] * R;
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < total;
       x += (long long)gridDim.x * blockDim.x) {
    long long rem = x;
    int k = 2;
    while (rem >= (long long)a.It[k - 2] * R) { rem -= (long long)a.It[k - 2] * R; ++k; }
    const int Ik = a.It[k - 2];
    const int i = (int)(rem % Ik), r = (int)(rem / Ik);
    const long long nother = a.Q / Ik;
    double s = 0.0;
    for (long long o = 0; o < nother; ++o) {
      long long oo = o, q = 0, stride = 1;
      double c = 1.0;
      for (int l = 2; l < a.N; ++l) {
        const int Il = a.It[l - 2];
        int il;
        if (l == k) {
          il = i;
        } else {
          il = (int)(oo % Il);
          oo /= Il;
          c *= a.A[a.off[l] + il + (long long)r * Il];
        }
        q += il * stride;
        stride *= Il;
      }
      s += tq[(long long)r * a.Q + q] * c;
    }
    M[a.off[k] + i + (long long)r * Ik] = s;
  }
}

__global__ void k_sum(const double* part, int n, double* out, const int* stop) {
  if (stopped(stop)) return;
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

template <typename TY>
__global__ void k_norm2(const TY* y, long long n, double* part) {
  __shared__ double red[16];
  double s = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const double a0 = to_f64(y[i]), a1 = to_f64(y[i + stride]);
    const double a2 = to_f64(y[i + 2 * stride]), a3 = to_f64(y[i + 3 * stride]);
    s += (a0 * a0 + a1 * a1) + (a2 * a2 + a3 * a3);
  }
  for (; i < n; i += stride) {
    const double v = to_f64(y[i]);
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace

PassPlan plan_pass(const Shape& s, YType yt) {
  PassPlan p{};
  p.tiles_i = (s.I[0] + 63) / 64;
  p.tiles_j = (s.I[1] + 63) / 64;
  p.Q = 1;
  for (int k = 2; k < s.N; ++k) p.Q *= s.I[k];
  const long long tiles = (long long)p.tiles_i * p.tiles_j;
  // MFMA passes: about one resident round (256 CUs x 2 blocks); a block walks
  // its q-chunk in sub-chunks of kQMax slabs
  const long long target = (yt != YType::F64) ? 512 : 2048;
  long long want = (target + tiles - 1) / tiles;
  if (want > p.Q) want = p.Q;
  if (want < 1) want = 1;
  p.q_per = (int)((p.Q + want - 1) / want);
  p.n_qc = (int)((p.Q + p.q_per - 1) / p.q_per);
  p.mfma = (yt != YType::F64) ? 1 : 0;
  p.tc_bytes = (yt == YType::F64) ? 8 : 4;
  p.m0_elems = (size_t)p.n_qc * p.tiles_j * s.R * s.I[0];
  p.m1_elems = (size_t)p.n_qc * p.tiles_i * s.R * s.I[1];
  p.t_elems = (size_t)tiles * s.R * p.Q;
  p.e2_elems = (size_t)tiles * p.n_qc;
  p.tbuf_elems = (s.N >= 4) ? (size_t)p.Q * s.R : 0;
  return p;
}

hipError_t launch_tensor_pass(const Shape& s, YType yt, const void* Y, const double* A, bool resid,
                              const PassPlan& p, const PassBuffers& b, double* M, double* e2out,
                              const int* stop, hipStream_t st, const PassFold* fold) {
  PassArgs a{};
  a.Y = Y;
  a.I0 = s.I[0];
  a.I1 = s.I[1];
  a.N = s.N;
  a.R = s.R;
  a.Q = p.Q;
  for (int k = 2; k < s.N; ++k) a.It[k - 2] = s.I[k];
  a.A = A;
  for (int k = 0; k < s.N; ++k) a.off[k] = s.off[k] * s.R;
  a.tiles_i = p.tiles_i;
  a.tiles_j = p.tiles_j;
  a.q_per = p.q_per;
  a.m0part = b.m0part;
  a.m1part = b.m1part;
  a.tpart = b.tpart;
  a.e2part = b.e2part;
  dim3 grid(p.tiles_i * p.tiles_j, p.n_qc);
  const int NB = (s.R + 15) / 16;
  if (yt == YType::F64) {
    if (resid) k_pass_fma<double, double, true><<<grid, 256, 0, st>>>(a, stop);
    else k_pass_fma<double, double, false><<<grid, 256, 0, st>>>(a, stop);
  } else if (yt == YType::F32) {
    // 16-byte pieces need I_1 % 4 == 0 and a 16-byte aligned tensor
    const bool vec = (s.I[0] % 4) == 0 && (reinterpret_cast<uintptr_t>(Y) % 16) == 0;
#define F32_CASE(nb)                                                                     \
  case nb:                                                                               \
    if (vec) {                                                                           \
      if (resid) k_pass_f32<nb, true, true><<<grid, 256, 0, st>>>(a, stop);              \
      else k_pass_f32<nb, false, true><<<grid, 256, 0, st>>>(a, stop);                   \
    } else {                                                                             \
      if (resid) k_pass_f32<nb, true, false><<<grid, 256, 0, st>>>(a, stop);             \
      else k_pass_f32<nb, false, false><<<grid, 256, 0, st>>>(a, stop);                  \
    }                                                                                    \
    break;
    switch (NB) { F32_CASE(1) F32_CASE(2) F32_CASE(3) F32_CASE(4) default: return hipErrorInvalidValue; }
#undef F32_CASE
  } else {
    if (resid) return hipErrorInvalidValue;  // the residual pass reads the FP32 tensor
    // 8-byte pieces need I_1 % 4 == 0 and an 8-byte aligned tensor
    const bool vec = (s.I[0] % 4) == 0 && (reinterpret_cast<uintptr_t>(Y) % 8) == 0;
#define BF16_CASE(nb)                                                      \
  case nb:                                                                 \
    if (vec) k_pass_bf16<nb, true><<<grid, 256, 0, st>>>(a, stop);         \
    else k_pass_bf16<nb, false><<<grid, 256, 0, st>>>(a, stop);            \
    break;
    switch (NB) { BF16_CASE(1) BF16_CASE(2) BF16_CASE(3) BF16_CASE(4) default: return hipErrorInvalidValue; }
#undef BF16_CASE
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nslot0 = p.n_qc * p.tiles_j, nslot1 = p.n_qc * p.tiles_i;
  const int ntile = p.tiles_i * p.tiles_j;
  const long long len0 = (long long)s.R * s.I[0], len1 = (long long)s.R * s.I[1];
  const long long lent = (long long)s.R * p.Q;
  double* tdst = (s.N == 3) ? M + (long long)s.off[2] * s.R : b.tbuf;
  ReduceArgs ra{};
  ra.seg[0] = SlotSeg{b.m0part, nslot0, len0, M + (long long)s.off[0] * s.R};
  ra.seg[1] = SlotSeg{b.m1part, nslot1, len1, M + (long long)s.off[1] * s.R};
  ra.seg[2] = SlotSeg{b.tpart, ntile, lent, tdst};
  for (int k = 0; k < 3; ++k) ra.nb[k] = (int)((ra.seg[k].len + 63) / 64);
  ra.A1 = A + (long long)s.off[0] * s.R;
  ra.N = s.N;
  ra.R2 = s.R * s.R;
  int nextra = 0;
  if (fold) {
    ra.ipart = fold->ipart;
    if (fold->rowpart) {
      ra.rowpart = fold->rowpart;
      ra.chunks = fold->chunks;
      ra.stride = fold->stride;
      ra.gout = fold->gout;
      ra.gscal = fold->gscal;
      nextra = s.N + 1;
    }
  }
  const unsigned nblk = (unsigned)(ra.nb[0] + ra.nb[1] + ra.nb[2] + nextra);
  if (p.tc_bytes == 8) k_reduce_slots<double><<<nblk, 1024, 0, st>>>(ra, stop);
  else k_reduce_slots<float><<<nblk, 1024, 0, st>>>(ra, stop);
  if (s.N >= 4) k_modes_from_t<<<256, 256, 0, st>>>(a, b.tbuf, M, stop);
  if (resid && e2out) k_sum<<<1, 256, 0, st>>>(b.e2part, (int)p.e2_elems, e2out, stop);
  return hipGetLastError();
}

hipError_t launch_norm2(YType yt, const void* Y, long long n, double* part, int nparts, double* out,
                        hipStream_t st) {
  if (yt == YType::F64) k_norm2<double><<<nparts, 256, 0, st>>>((const double*)Y, n, part);
  else if (yt == YType::F32) k_norm2<float><<<nparts, 256, 0, st>>>((const float*)Y, n, part);
  else k_norm2<__bf16><<<nparts, 256, 0, st>>>((const __bf16*)Y, n, part);
  k_sum<<<1, 256, 0, st>>>(part, nparts, out, nullptr);
  return hipGetLastError();
}

}  // namespace dgn
