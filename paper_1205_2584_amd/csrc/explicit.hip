// The plain damped Gauss-Newton step with an explicitly formed Hessian
// (Section 3): (J^T J + mu I) da = J^T vec(Y - Y_hat) with J^T J of size
// RT x RT, factored by the same tiled Cholesky as the fast step's trailing
// system (the gradient rides along as the right-hand-side row).  It is the
// dGN baseline of the paper's comparisons (Section 6), built here to compare
// cost and memory with the fast step; real tensors only.
#include "common.hpp"
#include "internal.hpp"

namespace dgn {

namespace {

// Parameter index q in the stacked factor layout (mode n occupies
// [off[n] R, off[n + 1] R), column-major I_n x R) -> mode n, row i, column r.
__device__ __forceinline__ void decode(const Shape& s, long long q, int& n, int& i, int& r) {
  n = 0;
  while (n + 1 < s.N && q >= (long long)s.off[n + 1] * s.R) ++n;
  const long long local = q - (long long)s.off[n] * s.R;
  i = (int)(local % s.I[n]);
  r = (int)(local / s.I[n]);
}

// Hadamard product of the Grams C^(k), k != skip1, skip2, entry (r, c).
__device__ __forceinline__ double gamma_at(const Shape& s, const double* C, int skip1, int skip2, int r, int c) {
  const int R2 = s.R * s.R;
  double g = 1.0;
  for (int k = 0; k < s.N; ++k)
    if (k != skip1 && k != skip2) g *= C[(long long)k * R2 + r + c * s.R];
  return g;
}

// H + mu I on the lower tiles and the gradient as the right-hand-side row
// (tile row Tt, its first row); padding rows and columns carry the identity.
// With a_n[i, r] the parameter of row (n, i, r) (Section 3 / Appendix B):
//   H[(n,i,r), (n,i',c)] = delta_ii' Gamma^(n)[r, c],
//   H[(n,i,r), (m,j,c)]  = A_n[i, c] A_m[j, r] Gamma^(n,m)[r, c]   (n != m).
__global__ __launch_bounds__(256) void k_hess_fill(Shape s, SysPlan p, const double* A, const double* C,
                                                   const double* G, double mu, double* St) {
  const long long nlow = (long long)p.Tt * (p.Tt + 1) / 2;
  const long long id = blockIdx.x;
  int ti, tj;
  if (id < nlow) {
    ti = (int)((sqrt(8.0 * id + 1.0) - 1.0) / 2.0);
    while ((long long)(ti + 1) * (ti + 2) / 2 <= id) ++ti;
    while ((long long)ti * (ti + 1) / 2 > id) --ti;
    tj = (int)(id - (long long)ti * (ti + 1) / 2);
  } else {
    ti = p.Tt;
    tj = (int)(id - nlow);
  }
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    const long long row = (long long)ti * 64 + ii, col = (long long)tj * 64 + jj;
    double v = 0.0;
    if (ti == p.Tt) {
      v = (ii == 0 && col < p.nt) ? G[col] : 0.0;
    } else if (row >= p.nt || col >= p.nt) {
      v = (row == col) ? 1.0 : 0.0;
    } else {
      int n, i, r, m, j, c;
      decode(s, row, n, i, r);
      decode(s, col, m, j, c);
      if (n == m) {
        v = (i == j) ? gamma_at(s, C, n, -1, r, c) : 0.0;
        if (row == col) v += mu;
      } else {
        v = A[(long long)s.off[n] * s.R + i + (long long)c * s.I[n]] *
            A[(long long)s.off[m] * s.R + j + (long long)r * s.I[m]] * gamma_at(s, C, n, m, r, c);
      }
    }
    St[row + col * p.lds] = v;
  }
}

// A_c = A + da; scal[0] = da^T (g + mu da), scal[1] = ||da||^2 (one block).
__global__ __launch_bounds__(1024) void k_explicit_update(long long nt, const double* A, const double* da,
                                                          const double* G, double mu, double* Ac, double* scal) {
  __shared__ double red[16];
  double den = 0.0, d2 = 0.0;
  for (long long q = threadIdx.x; q < nt; q += blockDim.x) {
    const double d = da[q];
    Ac[q] = A[q] + d;
    den += d * (G[q] + mu * d);
    d2 += d * d;
  }
  den = block_sum(den, red);
  d2 = block_sum(d2, red);
  if (threadIdx.x == 0) {
    scal[0] = den;
    scal[1] = d2;
  }
}

}  // namespace

SysPlan plan_sys_explicit(const Shape& s) {
  SysPlan p{};
  p.R2 = s.R * s.R;
  p.nt = s.R * s.T;
  p.ntp = ((p.nt + 63) / 64) * 64;
  p.Tt = p.ntp / 64;
  p.lds = p.ntp + 64;
  return p;
}

hipError_t launch_explicit_system(const Shape& s, const SysPlan& p, const double* A, const double* C,
                                  const double* G, double mu, double* St, hipStream_t st) {
  const long long blocks = (long long)p.Tt * (p.Tt + 1) / 2 + p.Tt;
  k_hess_fill<<<(unsigned)blocks, 256, 0, st>>>(s, p, A, C, G, mu, St);
  return hipGetLastError();
}

hipError_t launch_explicit_update(const SysPlan& p, const double* A, const double* da, const double* G,
                                  double mu, double* Ac, double* scal, hipStream_t st) {
  k_explicit_update<<<1, 1024, 0, st>>>(p.nt, A, da, G, mu, Ac, scal);
  return hipGetLastError();
}

}  // namespace dgn
