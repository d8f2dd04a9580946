// Shared device helpers and data structures of the gfx950 fLM library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgn {

constexpr int kWave = 64;
constexpr int kMaxOrder = 8;
constexpr int kMaxRank = 64;
constexpr int kTile = 64;  // tile edge of the dense NR^2 system and of the tensor pass

// Shape of one CP problem.  Factors of all modes are stacked: mode n occupies
// a column-major I_n x R block starting at element off[n] * R.
struct Shape {
  int N, R;
  int I[kMaxOrder];
  int off[kMaxOrder];
  int T;     // sum of I_n
  int maxI;
};

// Device-resident state of a fit (Algorithm 1 with the damping of Section 4.5).
struct FitState {
  double mu, mu0, err2, err2_cand, denom, rho;
  double ynorm2;       // ||Y||^2 of the master tensor (relative error)
  double ynorm2_pass;  // ||Y||^2 of the tensor read by the plain passes
  double eps, eps_prev, tol;
  double gnorm2, danorm2, mnorm2;
  int iters, accepted, stop, reason;
  int max_iters, commit_iter, singular, normalize;
  int resid, resid_iters, pad0, mu_rule;  // mu_rule: 0 double on a rejection, 1 Nielsen's nu rule
  double cg_mu_fail;   // damping of the trial whose CG solve did not converge (0: none yet)
  double nu;           // growth factor of the next rejection under Nielsen's rule
  long long t0_ticks, t1_ticks;  // batched fits: device clock at the initial state and at the stop
  double scale[kMaxOrder * kMaxRank];  // column scales of the last normalisation
};

__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(__bf16 x) { return (float)x; }
__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(float x) { return (double)x; }
__device__ __forceinline__ double to_f64(__bf16 x) { return (double)(float)x; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Workgroup barrier.  On gfx950 s_barrier does not wait for the wave's own
// outstanding LDS operations, so a barrier that orders LDS accesses between
// waves has to be preceded by s_waitcnt lgkmcnt(0).  __syncthreads() gets that
// wait from its release fence, but hipcc (ROCm 7.2) has been seen to drop it on
// some paths into a barrier (a loop back-edge, a branch around the last LDS
// store), leaving a store or load in flight while other waves pass the barrier.
// The explicit wait here is an ordinary s_waitcnt, which the compiler keeps:
// immediate 0xC07F = lgkmcnt(0) with the vmcnt and expcnt fields at their maxima.
__device__ __forceinline__ void sync_block() {
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __syncthreads();
}

// Block-wide sum for blockDim.x a multiple of 64 and <= 1024; every thread gets the result.
template <typename T>
__device__ T block_sum(T v, T* scratch /* >= 16 entries of shared memory */) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  sync_block();
  if (l == 0) scratch[w] = v;
  sync_block();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  sync_block();
  return s;
}

__device__ __forceinline__ bool stopped(const int* stop) { return stop != nullptr && *stop != 0; }

}  // namespace dgn
