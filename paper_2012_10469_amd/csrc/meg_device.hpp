// Device-side data structures and helpers of the low-rank MEG library (gfx950).
//
// Layout in HBM (per context):
//   Qw   n x k  row-major, stride k: the warm-start basis; its first r columns
//               are V of the factored iterate X_t = alpha I + V diag(d) V^T
//   Za,Zb n x k ping-pong outputs of the operator apply, same layout
//   g    nnz    gradient values on Omega (masked objective)
//   Ctl  one control block (FP64 scalars and k x k transforms)
//   Red  partial sums of the per-workgroup Gram matrices
// Rows are 64 B (k = 16, float) or 128 B apart, so a row is read by one
// aligned vector load per lane group and Gram partials stay row-local.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace meg {

constexpr int KMAX = 32;

// Objective kinds (mirror meg_grad_kind).
enum Kind : int32_t { LINEAR_DENSE = 0, DENOISE_DENSE = 1, LINEAR_CSR = 2, MASKED_CSR = 3, QUADMEAS = 4 };

// Immutable per-context configuration, passed by value to every kernel.
struct Cfg {
  int64_t n;
  int64_t ld;    // dense leading dimension (elements)
  int64_t nnz;   // CSR entries
  int64_t lda;   // QUADMEAS pool row stride
  int64_t m;     // QUADMEAS pool size
  int64_t batch_steps;
  int32_t r, k, kind, prec;
  int32_t min_inner, max_inner, batch, pad;
  double eta, eps_scale, eps_c, eps_pow;
  double inner_tol;   // relative Ritz residual tolerance (top r pairs)
  double unit_round;  // 2^-24 (float state) or 2^-53 (double state)
  double cert_tol;    // absolute residual tolerance of the (r+1)-th pair (0: none)
};

// Step record copied back to the host (mirrors meg_step_info).
struct Info {
  int64_t t;
  double f, eps_t, cert_L, cert_bound;
  int32_t cert_holds, inner_iters;
  double ritz_gap, resid_max, mu_r1, sigma;
  int32_t converged, reserved;
  double resid_r1;
};

// Device control block: everything the step kernels exchange.
struct Ctl {
  double W[KMAX * KMAX];    // Q = Zin W is the (implicit, orthonormal) sweep basis
  double Pin[KMAX * KMAX];  // V^T Zin (r x k, row l, column b)
  double Wfin[KMAX * KMAX]; // final transform: Qw_next = Zsrc Wfin
  double theta[KMAX];       // Ritz values of the last Rayleigh-Ritz
  double resid[KMAX];       // Ritz residual norms
  double d[KMAX];           // X_t = alpha I + V diag(d) V^T
  double c[KMAX];           // log(alpha + d) - log(alpha)
  double ceff[KMAX];        // Yhat = V diag(ceff) V^T + opscale*Op + sdiag*I
  double alpha;
  double sdiag, opscale, sigma, gmax;
  double data_norm;         // ||M||_F, ||C||_F or ||vals||_2 (set once)
  double op_lmin, op_lmax;  // bounds on the extreme eigenvalues of the data
                            // operator (C, M or P_Omega(M)), set once (Lanczos)
  double f;                 // objective at X_t (when evaluated)
  double solve_tol;         // certificate bound at which meg_solve stops
  int64_t t;                // current iteration index (X_t)
  int32_t done;             // inner solve of this step finished
  int32_t sweep;            // next sweep index (1-based)
  int32_t src;              // buffer holding the input of the final sweep
  int32_t stop;             // meg_solve reached its tolerance: skip work
  int32_t status;           // 0 ok, else a meg_status code (sticky)
  int32_t fvalid;
  int32_t polish;           // extra sweeps taken after reaching the residual floor
  int32_t pad_;
  Info info;
};

// Two-level deterministic reduction workspace ("last workgroup" tree).
struct Red {
  double* part;     // nwg x plen
  double* gpart;    // ngroups x plen
  unsigned* cnt;    // ngroups + 1 arrival counters (zero between launches)
  int nwg, gsz, ngroups, plen;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Agent-scope arrival counter (global memory atomic, vector memory path).
__device__ __forceinline__ unsigned arrive(unsigned* c) {
  return __hip_atomic_fetch_add(c, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void reset_counter(unsigned* c) {
  __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every workgroup contributes `plen` doubles (in LDS `mine`).  Returns true in
// exactly one workgroup (the last to arrive), whose LDS `out` then holds the
// sum over all workgroups, added in a fixed order (bitwise reproducible).
// `out` may alias `mine`.  All threads of the workgroup must call this.
template <int NT>
__device__ bool tree_reduce(const Red& red, const double* mine, double* out) {
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int wg = blockIdx.x;
  const int plen = red.plen;
  double* dst = red.part + (size_t)wg * plen;
  for (int e = tid; e < plen; e += NT) dst[e] = mine[e];
  __threadfence();
  __syncthreads();
  const int g = wg / red.gsz;
  const int g0 = g * red.gsz;
  const int gn = min(red.gsz, red.nwg - g0);
  if (tid == 0) s_last = (arrive(&red.cnt[g]) == (unsigned)(gn - 1));
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double* gdst = red.gpart + (size_t)g * plen;
  for (int e = tid; e < plen; e += NT) {
    double s = 0.0;
    for (int w = 0; w < gn; ++w) s += red.part[(size_t)(g0 + w) * plen + e];
    gdst[e] = s;
  }
  if (tid == 0) reset_counter(&red.cnt[g]);
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = (arrive(&red.cnt[red.ngroups]) == (unsigned)(red.ngroups - 1));
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  for (int e = tid; e < plen; e += NT) {
    double s = 0.0;
    for (int q = 0; q < red.ngroups; ++q) s += red.gpart[(size_t)q * plen + e];
    out[e] = s;
  }
  if (tid == 0) reset_counter(&red.cnt[red.ngroups]);
  __syncthreads();
  return true;
}

__device__ __forceinline__ double eps_at(const Cfg& cfg, int64_t t) {
  return cfg.eps_scale / pow((double)t + cfg.eps_c + 1.0, cfg.eps_pow);
}

}  // namespace meg
