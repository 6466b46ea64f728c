// Device-side data structures and helpers of the low-rank MEG library (gfx950).
//
// Layout in HBM (per context):
//   Z0,Z1,Z2 n x k row-major, stride k: three blocks.  One of them (index
//               ctl->src) holds B, the warm-start basis in implicit form:
//               Q_t = B Wb is orthonormal and V = Q_t[:, :r] is V of the
//               factored iterate X_t = alpha I + V diag(d) V^T; the other two
//               take the outputs of the operator applies in turn
//   g    nnz    gradient values on Omega (masked objective)
//   Ctl  one control block (FP64 scalars and k x k transforms)
//   Bufs per-workgroup partial sums (FP64), their reduction, barrier words
// Rows are 64 B (k = 16, float) or 128 B apart, so a row is read by one
// aligned vector load per lane group and Gram partials stay row-local.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace meg {

constexpr int KMAX = 32;
constexpr int kMaxBatch = 1024;  // largest minibatch of the factored gradient

// Pointer into LDS.  The explicit address space lets functions that are not
// inlined into the kernel use LDS instructions; through a generic pointer
// they would use flat accesses, which are slower.
template <typename T>
using lds = __attribute__((address_space(3))) T;
// Pointer into global memory, for the same reason (flat accesses also wait
// on both the vector-memory and the LDS counters).
template <typename T>
using gbl = __attribute__((address_space(1))) T;

// Objective kinds (mirror meg_grad_kind).
enum Kind : int32_t { LINEAR_DENSE = 0, DENOISE_DENSE = 1, LINEAR_CSR = 2, MASKED_CSR = 3, QUADMEAS = 4, EXTERNAL = 5 };

// Immutable per-context configuration, passed by value to every kernel.
struct Cfg {
  int64_t n;
  int64_t ld;    // dense leading dimension (elements)
  int64_t nnz;   // CSR entries
  int64_t lda;   // QUADMEAS pool row stride
  int64_t m;     // QUADMEAS pool size
  int64_t batch_steps;
  int32_t r, k, kind, prec;
  int32_t min_inner, max_inner, batch;
  int32_t rr_from;    // first sweep with Rayleigh-Ritz (earlier sweeps only orthonormalise)
  double eta, eps_scale, eps_c, eps_pow;
  double inner_tol;   // relative Ritz residual tolerance (top r pairs)
  double unit_round;  // 2^-24 (float state) or 2^-53 (double state)
  double cert_tol;    // (r+1)-th pair: > 0 always resolve it to this absolute residual;
                      // 0 resolve it (to the top pairs' tolerance) whenever the
                      // certificate's lower bound could pass a decision; < 0 never
  // CSR kinds: each workgroup keeps its rows' slice of the sparse data in
  // dynamic LDS (0: disabled, the data is read from global memory)
  int32_t cache_blocks;  // row blocks per workgroup the cache holds
  int32_t cache_nnz;     // stored entries per workgroup the cache holds
  // explicit Ritz residuals (FP64 state): every Rayleigh-Ritz sweep's residual
  // block Zout S - Zin W S Theta is formed by the next sweep's apply, one
  // pass over its rows, instead of being estimated from Gram matrices only
  int32_t xres;
  // FP32 forms: a step may end on the block one power step past its last
  // Rayleigh-Ritz sweep when the residuals predict convergence (small_sweep)
  int32_t extrap;
  int32_t cheb;  // Chebyshev-filtered sweeps (interval [0, theta_k])
  int32_t pad2_;
};

// Byte offsets of the per-workgroup CSR cache in dynamic LDS:
//   rloc int[cache_blocks * (rows + 1)]  row starts, as positions in the cache
//   col  int[cache_nnz]                  column indices
//   val  T[cache_nnz]                    values (M_Omega or C)
//   g    T[cache_nnz]                    gradient values (masked objective)
struct CacheLayout {
  int64_t rloc, col, val, g, bytes;
};
__host__ __device__ inline int64_t align16(int64_t x) { return (x + 15) & ~(int64_t)15; }
__host__ __device__ inline CacheLayout cache_layout(int blocks, int rows, int nnz, int esize, bool with_g) {
  CacheLayout L;
  L.rloc = 0;
  L.col = align16((int64_t)blocks * (rows + 1) * 4);
  L.val = align16(L.col + (int64_t)nnz * 4);
  L.g = align16(L.val + (int64_t)nnz * esize);
  L.bytes = with_g ? align16(L.g + (int64_t)nnz * esize) : L.g;
  return L;
}

// Step record copied back to the host (mirrors meg_step_info).
struct Info {
  int64_t t;
  double f, eps_t, cert_L, cert_bound;
  int32_t cert_holds, inner_iters;
  double ritz_gap, resid_max, mu_r1, sigma;
  int32_t converged, cert_resolved;
  double resid_r1;
  double cert_L_up, mu_r1_up;
};

// Device control block: everything the step kernels exchange.
struct Ctl {
  double W[KMAX * KMAX];    // Q = Zin W is the (implicit, orthonormal) basis of the current sweep
  double PW[KMAX * KMAX];   // V^T Q = V^T Zin W (r x k, row l, column b)
  double Wb[KMAX * KMAX];   // basis transform: Q_t = B Wb, B = block `src`
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
  int32_t src;              // block holding B
  int32_t stop;             // meg_solve reached its tolerance: skip work
  int32_t status;           // 0 ok, else a meg_status code (sticky)
  int32_t fvalid;
  int32_t polish;           // extra sweeps taken after reaching the residual floor
  int32_t pxvalid;          // pxnorm holds ||P_Omega X_t||_F of the current t
  double pxnorm;            // ||P_Omega X_t||_F measured in sweep 1 (masked objective)
  double dxnorm;            // ||X_{t+1} - X_t||_F of the last step
  int64_t iters_done;       // iterations performed by step launches (counter)
  int64_t applies_done;     // operator applies performed by step launches (counter)
  int64_t jacobi_done;      // Jacobi sweeps of the Rayleigh-Ritz solves (counter)
  int64_t pause_seq;        // batched launches: the launch whose time budget this instance used up
  // explicit residuals (Cfg::xres): the last Rayleigh-Ritz sweep's sorted
  // Ritz vectors S and W S Theta, valid while xvalid is set (the next sweep's
  // apply forms Zin' S - Zin (W S Theta) with Zin' = that sweep's output)
  double XS[KMAX * KMAX];
  double XWT[KMAX * KMAX];
  int32_t xvalid;
  int32_t pad_;
  // an upper bound of mu_{r+1} for the step of iteration mu_up_t, from the
  // deflated Lanczos run of meg_certificate_bound (mu_up_t = 0: none)
  double mu_up;
  int64_t mu_up_t;
  int64_t extrap_done;  // steps that ended extrapolated (counter)
  int64_t unconv_done;  // steps whose inner solve hit max_inner unconverged (counter)
  // Chebyshev filter of the current sweep: the upper end b of the interval
  // [0, b] taken to hold the unwanted spectrum of Yhat (0: none, a plain
  // power step); the sweep outputs Zout = (Yhat - b/2) Q / (b/2)
  double cheb_b;
  double xscale;  // explicit residuals: 1 / |fa| of the sweep whose pairs they test
  // the ended step's eigenvalues mu_1 and mu_k of M_t (Ritz values), from
  // which the next step's first interval is taken (mu_valid = 0: none)
  double mu_1, mu_k;
  int32_t mu_valid;
  int32_t pad3_;
  double da_lmin;  // dual-averaging reading: a lower bound of lambda_min(Y_t)
  Info info;
};

// Scratch of the persistent step kernel: per-workgroup partial sums, their
// reduction, and the grid barrier words.
// Longest per-workgroup partial record of any step kernel (Gram matrices,
// the masked objective's two sums, the explicit residuals' column sums).
constexpr int kPartMax = 3 * KMAX * KMAX + 2 + KMAX;

// The record a sweep reduces over the grid (FP64), for block width KB and
// rank r, with Zout the sweep's output and Zin its input:
//   [0, KB^2)            C = Zin^T Zout
//   [KB^2, KB^2 + KT)    G = Zout^T Zout, upper triangle by rows
//   [KB^2 + KT, f)       P = V^T Zout, its r rows (V = the iterate's basis)
//   f, f + 1             the masked objective's sum of g^2 and of X_ij^2
//   f + 2 ...            (FP64 state) the explicit residuals' column sums
// G travels as a triangle and P without its zero rows: the barrier's
// reduction reads every word of every workgroup's record.
template <int KB>
struct PartRec {
  static constexpr int KT = KB * (KB + 1) / 2;
  static constexpr int G_OFF = KB * KB;
  static constexpr int P_OFF = KB * KB + KT;
  // position of (a, c), a <= c, in a triangle
  __host__ __device__ static constexpr int tri(int a, int c) { return a * KB - a * (a - 1) / 2 + (c - a); }
  __host__ __device__ static constexpr int f_off(int r) { return P_OFF + r * KB; }
  __host__ __device__ static constexpr int x_off(int r) { return f_off(r) + 2; }
  __host__ __device__ static constexpr int len(int r, bool xres) { return x_off(r) + (xres ? KB : 0); }
};
static_assert(PartRec<KMAX>::len(KMAX - 1, true) <= kPartMax, "partial record buffers");

struct Bufs {
  double* part;     // (workgroups of the team) x plen partial sums (FP64)
  double* gpart;    // per-barrier-group sums of the partials (FP64)
  double* sums;     // plen reduced sums
  unsigned* bar;    // barrier words, one 128-byte line each (see grid_sync)
  long long* ts;    // optional phase timestamps (wall clock), or null
};

// Barrier word layout (in unsigned units; 32 = one 128-byte line):
//   bar[0]            top-level arrival count
//   bar[32]           generation
//   bar[64]           error flag
//   bar[96 + 32 g]    arrival count of group g
constexpr int kBarTop = 0, kBarGen = 32, kBarErr = 64, kBarGroup0 = 96, kBarStride = 32;
constexpr int kBarGroupSize = 16;
constexpr int kBarMaxGroups = 64;  // up to 1024 workgroups
constexpr int kBarWords = kBarGroup0 + kBarStride * kBarMaxGroups;

// Phase timestamps (device wall clock) of a profiled launch: slots
// [0, kTsWg) are stamped by one workgroup at phase boundaries; from kTsWg on,
// every workgroup stamps the start of sweeps 1-2 and its arrival at their
// barriers: ts[kTsWg + (2 (s - 1) + e) * nwg + wg], e = 0 start, 1 arrival.
constexpr int kTsRR = 140;  // 5 slots: parts of the first Rayleigh-Ritz sweep
constexpr int kTsWg = 160;
constexpr int kTsWgSweeps = 2;
constexpr int kTsTotal = kTsWg + 2 * kTsWgSweeps * kBarGroupSize * kBarMaxGroups;

// Wavefront reductions (all 64 lanes active).  Within each row of 16 lanes
// four DPP exchanges combine lane pairs, quads, the two quads of a half-row
// (half-row mirror) and the two halves of the row (row mirror); both
// partners of every exchange compute the same value.  The four row results
// are then read as scalars and combined in a fixed order, so every lane gets
// the same, run-to-run reproducible result.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, dpp_f64<0xB1>(v));   // quad_perm [1, 0, 3, 2]: lane ^ 1
  v = op(v, dpp_f64<0x4E>(v));   // quad_perm [2, 3, 0, 1]: lane ^ 2
  v = op(v, dpp_f64<0x141>(v));  // row_half_mirror
  v = op(v, dpp_f64<0x140>(v));  // row_mirror
  return op(op(lane_f64(v, 0), lane_f64(v, 16)), op(lane_f64(v, 32), lane_f64(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, [](double a, double b) { return fmin(a, b); });
}

// Bounded spin: a barrier that is never completed (which a co-resident,
// cooperatively launched grid rules out) ends with the error flag set
// instead of a hang.
constexpr unsigned kSpinLimit = 1u << 22;

// Partial-sum elements per thread whose loads the barrier's reductions issue
// together (a per-workgroup record of up to kRedU * NT doubles is reduced in
// one round of loads).
constexpr int kRedU = 2;

// The two reduction levels of grid_sync (below), kept out of line so their
// loads in flight do not add to the register pressure of the caller.
// Group level: gpart[g] = sum over the group's workgroups w of part[w], in
// workgroup order; kRedU elements per thread have their loads issued together.
// Barrier order of the workgroups of a team.  A grid launched on all
// compute units places workgroup w on XCD w % 8; with a multiple of 8
// workgroups the barrier enumerates them XCD by XCD (position
// p = (w % 8) (P / 8) + w / 8), so each arrival group of kBarGroupSize
// holds workgroups of one XCD, whose partials sit in that XCD's L2.
__device__ __forceinline__ unsigned bar_pos(unsigned w, unsigned P, bool xcd) {
  return xcd ? (w % 8u) * (P / 8u) + w / 8u : w;
}
__device__ __forceinline__ unsigned bar_wg(unsigned pos, unsigned P, bool xcd) {
  return xcd ? (pos % (P / 8u)) * 8u + pos / (P / 8u) : pos;
}

template <int NT>
__device__ __noinline__ void reduce_group(const gbl<double>* part, gbl<double>* gpart, int plen, unsigned g,
                                          unsigned g0, unsigned gsize, unsigned P, bool xcd) {
  for (int e0 = threadIdx.x; e0 < plen; e0 += NT * kRedU) {
    double v[kRedU][kBarGroupSize];
#pragma unroll
    for (int u = 0; u < kRedU; ++u)
#pragma unroll
      for (int w = 0; w < kBarGroupSize; ++w) {
        const int e = e0 + u * NT;
        v[u][w] = (w < (int)gsize && e < plen) ? part[(size_t)bar_wg(g0 + w, P, xcd) * plen + e] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < kRedU; ++u) {
      const int e = e0 + u * NT;
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kBarGroupSize; ++w) s += v[u][w];
      if (e < plen) gpart[(size_t)g * plen + e] = s;
    }
  }
}

// Top level: sums = sum over the ng groups of gpart, in group order (sums
// in global memory or in the workgroup's LDS).
template <int NT, typename DP>
__device__ __noinline__ void reduce_top(const gbl<double>* gpart, DP sums, int plen, unsigned ng) {
  for (int e0 = threadIdx.x; e0 < plen; e0 += NT * kRedU) {
    double s[kRedU];
#pragma unroll
    for (int u = 0; u < kRedU; ++u) s[u] = 0.0;
    for (unsigned q0 = 0; q0 < ng; q0 += 16) {
      double v[kRedU][16];
#pragma unroll
      for (int u = 0; u < kRedU; ++u)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = e0 + u * NT;
          v[u][q] = (q0 + q < ng && e < plen) ? gpart[(size_t)(q0 + q) * plen + e] : 0.0;
        }
#pragma unroll
      for (int u = 0; u < kRedU; ++u)
#pragma unroll
        for (int q = 0; q < 16; ++q) s[u] += v[u][q];
    }
#pragma unroll
    for (int u = 0; u < kRedU; ++u)
      if (e0 + u * NT < plen) sums[e0 + u * NT] = s[u];
  }
}

// The workgroups that run one instance: this workgroup's rank and their
// count.  A single-instance launch is one team (blockIdx.x, gridDim.x); the
// batched kernel splits its grid into one team per resident instance.
struct Team {
  int wg, nwg;
  bool xcd = false;  // whole grid: arrival groups by XCD (bar_pos)
};
__device__ __forceinline__ Team grid_team() {
  return Team{(int)blockIdx.x, (int)gridDim.x, gridDim.x % 8u == 0 && gridDim.x >= 16u};
}

// Barrier over one team of a cooperatively launched grid (<= 1024 workgroups).
// Arrivals are counted in two levels (groups of kBarGroupSize workgroups,
// then the groups) so that no counter sees more than ~32 contending atomics.
// Every workgroup's writes before the barrier are visible to every workgroup
// after it: each arrival is an agent-scope acquire-release RMW (the group's
// last arriver carries the group's writes on to the top counter), and waiting
// workgroups acquire after observing the new generation.  `serial` runs in the
// last workgroup to arrive, with all of its threads, before anyone is
// released; its writes are published by the generation bump.  Returns false
// on a barrier error.
// With plen > 0 the barrier also sums the per-workgroup partials
// part[w * plen + e] into sums[e] on its way up the arrival tree: the last
// arriver of each group adds its group's partials (in workgroup order) into
// gpart, the last group adds the group sums (in group order).  The order is
// fixed, so the sums are bitwise reproducible.  All threads call it.
// A serial part that returns an int passes thread 0's value, a tag in [0, 8), to every
// workgroup of the team through the generation word itself (the last
// arrival advances it by 1 + 8 tag), so no workgroup reads it back from
// memory: *tag receives it (0 for a serial part that returns nothing).
// With lsums (LDS of the calling workgroup) the sums go there instead of to
// b.sums: only the workgroup that runs `serial` holds them, with no global
// write and read-back between the reduction and the serial part.
template <int NT, typename F>
__device__ __forceinline__ bool grid_sync(const Bufs& b, Team tm, int plen, F&& serial, int* tag = nullptr,
                                          lds<double>* lsums = nullptr) {
  __shared__ int s_role;  // 0: plain arrival, 1: last of its group, 2: last overall
  __shared__ unsigned s_gen;
  __shared__ int s_ok;
  __shared__ int s_tag;
  const int tid = threadIdx.x;
  auto run_serial = [&]() -> int {
    if constexpr (std::is_void<decltype(serial())>::value) {
      serial();
      return 0;
    } else {
      return serial();
    }
  };
  if (tm.nwg == 1) {  // a team of one workgroup: its partials are the sums
    __syncthreads();
    if (plen > 0 && lsums) {
      for (int e = tid; e < plen; e += NT) lsums[e] = b.part[e];
      __syncthreads();
    } else if (plen > 0 && b.sums != b.part) {
      for (int e = tid; e < plen; e += NT) b.sums[e] = b.part[e];
      __syncthreads();
    }
    const int tg = run_serial();
    if (tid == 0) s_tag = tg;  // thread 0's value is the tag, as below
    __syncthreads();
    if (tag) *tag = s_tag;
    return true;
  }
  const unsigned P = (unsigned)tm.nwg;
  const unsigned g = bar_pos((unsigned)tm.wg, P, tm.xcd) / kBarGroupSize;
  const unsigned ng = (P + kBarGroupSize - 1) / kBarGroupSize;
  const unsigned g0 = g * kBarGroupSize;
  const unsigned gsize = min((unsigned)kBarGroupSize, P - g0);
  unsigned* gc = &b.bar[kBarGroup0 + kBarStride * g];
  __syncthreads();
  if (tid == 0) {
    s_role = 0;
    // the error flag and the generation are read together
    const unsigned err = __hip_atomic_load(&b.bar[kBarErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned gen = __hip_atomic_load(&b.bar[kBarGen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_ok = err == 0;
    s_gen = gen;
    if (s_ok) {
      const unsigned prev = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == gsize - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the group's writes
        __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_role = 1;
      }
    }
  }
  __syncthreads();
  if (!s_ok) return false;
  if (s_role >= 1) {
    if (plen > 0) {
      reduce_group<NT>((const gbl<double>*)b.part, (gbl<double>*)b.gpart, plen, g, g0, gsize, P, tm.xcd);
      __syncthreads();
    }
    if (tid == 0) {
      const unsigned top = __hip_atomic_fetch_add(&b.bar[kBarTop], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (top == ng - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every group's writes
        s_role = 2;
      }
    }
    __syncthreads();
  }
  if (s_role == 2) {
    if (plen > 0) {
      if (lsums)
        reduce_top<NT>((const gbl<double>*)b.gpart, lsums, plen, ng);
      else
        reduce_top<NT>((const gbl<double>*)b.gpart, (gbl<double>*)b.sums, plen, ng);
      __syncthreads();
    }
    const int tg = run_serial();  // uniform over the workgroup
    __syncthreads();
    if (threadIdx.x == 0) {
      s_tag = tg;
      __hip_atomic_store(&b.bar[kBarTop], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&b.bar[kBarGen], 1u + 8u * (unsigned)tg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (tid == 0) {
    unsigned spins = 0, gen;
    while ((gen = __hip_atomic_load(&b.bar[kBarGen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == s_gen) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit || __hip_atomic_load(&b.bar[kBarErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_fetch_or(&b.bar[kBarErr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_ok = 0;
        break;
      }
    }
    s_tag = (int)(((gen - s_gen) - 1u) >> 3);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (tag) *tag = s_tag;
  return s_ok != 0;
}

template <int NT>
__device__ __forceinline__ bool grid_sync(const Bufs& b, Team tm) {
  return grid_sync<NT>(b, tm, 0, [] {});
}

__device__ __forceinline__ double eps_at(const Cfg& cfg, int64_t t) {
  return cfg.eps_scale / pow((double)t + cfg.eps_c + 1.0, cfg.eps_pow);
}

}  // namespace meg
