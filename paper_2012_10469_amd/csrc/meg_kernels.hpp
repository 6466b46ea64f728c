// HIP kernels of one low-rank MEG step (gfx950, wave64).
//
// Step t (Algorithm 2, Section 3):
//   grad  : gradient values of the masked objective on Omega at X_t, f(X_t),
//           ||grad||_F  (the last workgroup sets the step's shift)
//   apply : Zout = Yhat (Zin W) for the implicit orthonormal basis Q = Zin W,
//           Yhat = V diag(ceff) V^T + opscale * Op + sdiag * I, with the
//           Gram partials Zin^T Zout, Zout^T Zout, V^T Zout fused into the
//           epilogue; the last workgroup runs Rayleigh-Ritz + Cholesky QR
//   final : Qw <- Zsrc Wfin (Ritz basis = next warm start, first r columns =
//           V_{t+1}) and its Gram, whose Cholesky factor orthonormalises the
//           first sweep of the next step
// Launch shapes are fixed per problem size; kernels that find the inner solve
// finished (ctl->done) or the run stopped (ctl->stop) return immediately, so
// a step can be captured once as a graph of max_inner sweeps.
#pragma once
#include "meg_device.hpp"
#include "meg_small.hpp"

namespace meg {

// 16-byte vector of T (float4 / double2) used for row-chunk loads.
template <typename T> struct V16;
template <> struct V16<float> {
  static constexpr int N = 4;
  using type = float4;
};
template <> struct V16<double> {
  static constexpr int N = 2;
  using type = double2;
};

template <typename T>
__device__ __forceinline__ void vload(const T* p, T* out) {
  using VT = typename V16<T>::type;
  const VT v = *reinterpret_cast<const VT*>(p);
  if constexpr (V16<T>::N == 4) {
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
  } else {
    out[0] = v.x; out[1] = v.y;
  }
}

// Scratch doubles the last workgroup needs for the small solve.
template <int KB>
constexpr int small_scratch() { return 5 * KB * (KB + 1) + 8 * KB; }

__device__ __forceinline__ bool step_skipped(const Ctl* ctl) {
  return (ctl->stop | ctl->status) != 0;
}

// ---------------------------------------------------------------------------
// prep: step scalars for objectives without a gradient pass
// ---------------------------------------------------------------------------
__global__ void k_prep(Cfg cfg, Ctl* ctl) {
  if (step_skipped(ctl)) return;
  if (threadIdx.x == 0) {
    double gmax;
    if (cfg.kind == DENOISE_DENSE) {
      // lambda_max(X - M) <= lambda_max(X) - lambda_min(M), lambda_max(X) = alpha + max(0, max d)
      double dmax = 0.0;
      for (int l = 0; l < cfg.r; ++l) dmax = fmax(dmax, ctl->d[l]);
      gmax = ctl->alpha + dmax - ctl->op_lmin;
    } else {
      gmax = ctl->op_lmax;  // G = C
    }
    setup_step(cfg, ctl, gmax);
  }
}

// ---------------------------------------------------------------------------
// grad (masked CSR): g_e = X_ij - M_ij on Omega, f = 1/2 sum g^2
// X_ij = alpha [i == j] + sum_l V_il d_l V_jl.  One wave per row.
// ---------------------------------------------------------------------------
template <typename T, int KB>
__global__ __launch_bounds__(256) void k_grad_masked(Cfg cfg, Ctl* __restrict__ ctl, const int* __restrict__ rp,
                                                     const int* __restrict__ col, const T* __restrict__ mval,
                                                     const T* __restrict__ Qw, T* __restrict__ g, Red red) {
  if (step_skipped(ctl)) return;
  __shared__ T sd[KMAX];
  __shared__ double sred[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = cfg.r;
  if (tid < KMAX) sd[tid] = (T)ctl->d[tid];
  const T alpha = (T)ctl->alpha;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  double acc = 0.0, accx = 0.0;
  if (i < cfg.n) {
    T vi[KB];
#pragma unroll
    for (int l = 0; l < KB; ++l) vi[l] = (l < r) ? Qw[i * KB + l] * sd[l] : (T)0;
    const int e0 = rp[i], e1 = rp[i + 1];
    for (int e = e0 + lane; e < e1; e += 64) {
      const int j = col[e];
      const T* vj = Qw + (int64_t)j * KB;
      T x = (j == i) ? alpha : (T)0;
#pragma unroll
      for (int l = 0; l < KB; ++l)
        if (l < r) x += vi[l] * vj[l];
      const T gv = x - mval[e];
      g[e] = gv;
      acc += (double)gv * (double)gv;
      accx += (double)x * (double)x;
    }
  }
  acc = wave_sum(acc);
  accx = wave_sum(accx);
  if (lane == 0) {
    sred[wave] = acc;
    sred[4 + wave] = accx;
  }
  __syncthreads();
  __shared__ double mine[2];
  if (tid == 0) {
    mine[0] = sred[0] + sred[1] + sred[2] + sred[3];
    mine[1] = sred[4] + sred[5] + sred[6] + sred[7];
  }
  __syncthreads();
  if (tree_reduce<256>(red, mine, mine)) {
    if (tid == 0) {
      ctl->f = 0.5 * mine[0];
      ctl->fvalid = 1;
      // lambda_max(P(X) - P(M)) <= ||P(X)||_F - lambda_min(P(M)),  P = P_Omega
      setup_step(cfg, ctl, sqrt(mine[1]) - ctl->op_lmin);
    }
  }
}

// ---------------------------------------------------------------------------
// shared epilogue of the apply kernels
//   sU  : ROWS x KB row sums (Op Zin) for the workgroup's rows
//   out : Zout rows, plus Gram partials and (last workgroup) the small solve
// ---------------------------------------------------------------------------
template <typename T, int KB, int ROWS, int NT>
struct ApplySmem {
  static constexpr int LD = KB + 1;
  // typed section (in units of T)
  static constexpr int T_W = 0;                    // KB x LD
  static constexpr int T_P = T_W + KB * LD;        // KB x KB (r rows used)
  static constexpr int T_CE = T_P + KB * KB;       // KB
  static constexpr int T_ZIN = T_CE + KB;          // ROWS x KB
  static constexpr int T_V = T_ZIN + ROWS * KB;    // ROWS x KB
  static constexpr int T_U = T_V + ROWS * KB;      // ROWS x KB
  static constexpr int T_ZO = T_U + ROWS * KB;     // ROWS x KB
  static constexpr int T_END = T_ZO + ROWS * KB;
  static constexpr int TYPED_DOUBLES = (T_END * (int)sizeof(T) + 7) / 8;
  static constexpr int PLEN = 3 * KB * KB;
  static constexpr int SMALL = small_scratch<KB>();
  static constexpr int TOTAL = PLEN + (TYPED_DOUBLES > SMALL ? TYPED_DOUBLES : SMALL);
};

template <typename T, int KB, int ROWS, int NT>
__device__ void apply_prologue(const Cfg& cfg, const Ctl* ctl, T* tb, const T* __restrict__ Qw,
                               const T* __restrict__ Zin, int64_t row0) {
  using SM = ApplySmem<T, KB, ROWS, NT>;
  constexpr int LD = SM::LD;
  const int tid = threadIdx.x;
  const int r = cfg.r;
  for (int e = tid; e < KB * KB; e += NT) {
    tb[SM::T_W + (e / KB) * LD + (e % KB)] = (T)ctl->W[e];
    tb[SM::T_P + e] = (e / KB < r) ? (T)ctl->Pin[e] : (T)0;
  }
  if (tid < KB) tb[SM::T_CE + tid] = (T)ctl->ceff[tid];
  for (int e = tid; e < ROWS * KB; e += NT) {
    const int rr = e / KB, cc = e % KB;
    const int64_t i = row0 + rr;
    const bool ok = i < cfg.n;
    tb[SM::T_ZIN + e] = ok ? Zin[i * KB + cc] : (T)0;
    tb[SM::T_V + e] = (ok && cc < r) ? Qw[i * KB + cc] : (T)0;
  }
}

// Given sU (Op Zin rows), form Zout rows, store them and run the reduction.
template <typename T, int KB, int ROWS, int NT>
__device__ void apply_epilogue(const Cfg& cfg, Ctl* ctl, double* smem, T* __restrict__ Zout, int64_t row0,
                               const Red& red, int sweep, int in_buf) {
  using SM = ApplySmem<T, KB, ROWS, NT>;
  constexpr int LD = SM::LD;
  T* tb = reinterpret_cast<T*>(smem + SM::PLEN);
  const int tid = threadIdx.x;
  const int r = cfg.r;
  const T opscale = (T)ctl->opscale, sdiag = (T)ctl->sdiag;
  // u = opscale*(Op Zin)_i + V_i diag(ceff) Pin + sdiag Zin_i     (in the Zin basis)
  for (int e = tid; e < ROWS * KB; e += NT) {
    const int rr = e / KB, a = e % KB;
    T u = opscale * tb[SM::T_U + e] + sdiag * tb[SM::T_ZIN + e];
    for (int l = 0; l < r; ++l) u += tb[SM::T_V + rr * KB + l] * tb[SM::T_CE + l] * tb[SM::T_P + l * KB + a];
    tb[SM::T_ZO + e] = u;
  }
  __syncthreads();
  // z = u W, store, keep in LDS (zero rows beyond n)
  for (int e = tid; e < ROWS * KB; e += NT) {
    const int rr = e / KB, b = e % KB;
    T z = 0;
#pragma unroll 8
    for (int a = 0; a < KB; ++a) z += tb[SM::T_ZO + rr * KB + a] * tb[SM::T_W + a * LD + b];
    const int64_t i = row0 + rr;
    if (i < cfg.n) Zout[i * KB + b] = z; else z = 0;
    tb[SM::T_U + e] = z;  // reuse U for Zout rows
  }
  __syncthreads();
  // Gram partials in FP64 (products of working-precision values are exact)
  for (int e = tid; e < KB * KB; e += NT) {
    const int a = e / KB, b = e % KB;
    double c = 0.0, gg = 0.0, p = 0.0;
#pragma unroll 4
    for (int rr = 0; rr < ROWS; ++rr) {
      const double zb = (double)tb[SM::T_U + rr * KB + b];
      c += (double)tb[SM::T_ZIN + rr * KB + a] * zb;
      gg += (double)tb[SM::T_U + rr * KB + a] * zb;
      p += (double)tb[SM::T_V + rr * KB + a] * zb;
    }
    smem[e] = c;
    smem[KB * KB + e] = gg;
    smem[2 * KB * KB + e] = p;
  }
  __syncthreads();
  if (tree_reduce<NT>(red, smem, smem)) {
    small_sweep<KB, NT>(cfg, ctl, smem, smem + SM::PLEN, sweep, in_buf);
  }
}

// ---------------------------------------------------------------------------
// apply, CSR operator (masked gradient values g, or linear C values)
// ROWS rows per workgroup, one row per wave at a time.  A row's nonzeros are
// split over lane groups of LPN lanes; each lane owns a 16-byte column chunk
// of the gathered Zin row.
// ---------------------------------------------------------------------------
template <typename T, int KB, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_apply_csr(Cfg cfg, Ctl* __restrict__ ctl, const int* __restrict__ rp,
                                                  const int* __restrict__ col, const T* __restrict__ gv,
                                                  const T* __restrict__ Qw, const T* __restrict__ Zin,
                                                  T* __restrict__ Zout, Red red, int sweep, int in_buf) {
  if (ctl->done || step_skipped(ctl)) return;
  using SM = ApplySmem<T, KB, ROWS, NT>;
  __shared__ double smem[SM::TOTAL];
  T* tb = reinterpret_cast<T*>(smem + SM::PLEN);
  constexpr int VN = V16<T>::N;
  constexpr int LPN = KB / VN;       // lanes per nonzero
  constexpr int NPI = 64 / LPN;      // nonzeros per wave iteration
  constexpr int WAVES = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sub = lane % LPN, grp = lane / LPN;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  apply_prologue<T, KB, ROWS, NT>(cfg, ctl, tb, Qw, Zin, row0);
  for (int rr = wave; rr < ROWS; rr += WAVES) {
    const int64_t i = row0 + rr;
    T acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = 0;
    if (i < cfg.n) {
      const int e0 = rp[i], e1 = rp[i + 1];
      for (int e = e0 + grp; e < e1; e += NPI) {
        const int j = col[e];
        const T w = gv[e];
        T z[VN];
        vload<T>(Zin + (int64_t)j * KB + sub * VN, z);
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] += w * z[v];
      }
    }
#pragma unroll
    for (int o = LPN; o < 64; o <<= 1)
#pragma unroll
      for (int v = 0; v < VN; ++v) acc[v] += __shfl_xor(acc[v], o, 64);
    if (grp == 0) {
#pragma unroll
      for (int v = 0; v < VN; ++v) tb[SM::T_U + rr * KB + sub * VN + v] = acc[v];
    }
  }
  __syncthreads();
  apply_epilogue<T, KB, ROWS, NT>(cfg, ctl, smem, Zout, row0, red, sweep, in_buf);
}

// ---------------------------------------------------------------------------
// apply, dense operator (C or M, n x n row-major, leading dimension ld).
// Each wave owns RPW rows; the workgroup streams column chunks of 64 and
// stages the matching 64 rows of Zin in LDS once for all its rows.
// ---------------------------------------------------------------------------
template <typename T, int KB, int RPW, int NT>
__global__ __launch_bounds__(NT) void k_apply_dense(Cfg cfg, Ctl* __restrict__ ctl, const T* __restrict__ D,
                                                    const T* __restrict__ Qw, const T* __restrict__ Zin,
                                                    T* __restrict__ Zout, Red red, int sweep, int in_buf) {
  if (ctl->done || step_skipped(ctl)) return;
  constexpr int WAVES = NT / 64;
  constexpr int ROWS = RPW * WAVES;
  using SM = ApplySmem<T, KB, ROWS, NT>;
  __shared__ double smem[SM::TOTAL];
  __shared__ T zc[64][KB + 1];
  T* tb = reinterpret_cast<T*>(smem + SM::PLEN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = cfg.n;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  apply_prologue<T, KB, ROWS, NT>(cfg, ctl, tb, Qw, Zin, row0);
  T acc[RPW][KB];
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[q][c] = 0;
  for (int64_t j0 = 0; j0 < n; j0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * KB; e += NT) {
      const int jj = e / KB, c = e % KB;
      const int64_t j = j0 + jj;
      zc[jj][c] = (j < n) ? Zin[j * KB + c] : (T)0;
    }
    __syncthreads();
    const int64_t j = j0 + lane;
    T dv[RPW];
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const int64_t i = row0 + wave * RPW + q;
      dv[q] = (i < n && j < n) ? D[i * cfg.ld + j] : (T)0;
    }
#pragma unroll
    for (int c = 0; c < KB; ++c) {
      const T z = zc[lane][c];
#pragma unroll
      for (int q = 0; q < RPW; ++q) acc[q][c] += dv[q] * z;
    }
  }
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int c = 0; c < KB; ++c) {
      T v = acc[q][c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) tb[SM::T_U + (wave * RPW + q) * KB + c] = v;
    }
  __syncthreads();
  apply_epilogue<T, KB, ROWS, NT>(cfg, ctl, smem, Zout, row0, red, sweep, in_buf);
}

// ---------------------------------------------------------------------------
// finalize: Qw <- Zsrc Wfin, Gram of the new Qw, orthonormalising transform.
// mode 0: end of a step (advance t); mode 1: fresh basis (init / set_iterate).
// ---------------------------------------------------------------------------
template <typename T, int KB, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_finalize(Cfg cfg, Ctl* __restrict__ ctl, T* __restrict__ Qw,
                                                 const T* __restrict__ Za, const T* __restrict__ Zb, Red red,
                                                 int mode) {
  if (mode == 0 && (!ctl->done || ctl->status)) return;
  constexpr int LD = KB + 1;
  constexpr int PLEN = KB * KB;
  constexpr int SMALL = 2 * KB * LD + 64;
  __shared__ double smem[PLEN + SMALL];
  __shared__ T sWf[KB][LD];
  __shared__ T rows_in[ROWS][KB];
  __shared__ T rows_out[ROWS][KB];
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  const int src = (mode == 0) ? ctl->src : 0;
  const T* Zs = (src == 0) ? Qw : (src == 1 ? Za : Zb);
  for (int e = tid; e < KB * KB; e += NT)
    sWf[e / KB][e % KB] = (mode == 0) ? (T)ctl->Wfin[e] : (T)((e / KB) == (e % KB));
  for (int e = tid; e < ROWS * KB; e += NT) {
    const int64_t i = row0 + e / KB;
    rows_in[e / KB][e % KB] = (i < cfg.n) ? Zs[i * KB + e % KB] : (T)0;
  }
  __syncthreads();
  for (int e = tid; e < ROWS * KB; e += NT) {
    const int rr = e / KB, b = e % KB;
    T z = 0;
#pragma unroll 8
    for (int a = 0; a < KB; ++a) z += rows_in[rr][a] * sWf[a][b];
    const int64_t i = row0 + rr;
    if (i < cfg.n) Qw[i * KB + b] = z; else z = 0;
    rows_out[rr][b] = z;
  }
  __syncthreads();
  for (int e = tid; e < KB * KB; e += NT) {
    const int a = e / KB, b = e % KB;
    double s = 0.0;
#pragma unroll 4
    for (int rr = 0; rr < ROWS; ++rr) s += (double)rows_out[rr][a] * (double)rows_out[rr][b];
    smem[e] = s;
  }
  __syncthreads();
  if (tree_reduce<NT>(red, smem, smem)) {
    basis_setup<KB, NT>(cfg, ctl, smem, smem + PLEN);
    if (tid == 0 && mode == 0) ctl->t = ctl->t + 1;
    if (tid == 0) ctl->fvalid = 0;
  }
}

// ---------------------------------------------------------------------------
// objective at X_t, dense kinds: LINEAR sum C_ij X_ij, DENOISE 1/2 sum (X_ij - M_ij)^2
// X_ij = alpha [i == j] + sum_l V_il d_l V_jl, accumulated in FP64.
// One wave per row.
// ---------------------------------------------------------------------------
template <typename T, int KB>
__global__ __launch_bounds__(256) void k_objective_dense(Cfg cfg, Ctl* __restrict__ ctl, const T* __restrict__ D,
                                                         const T* __restrict__ Qw, Red red) {
  __shared__ double sd[KMAX];
  __shared__ double sred[4];
  __shared__ double mine[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = cfg.r;
  if (tid < KMAX) sd[tid] = ctl->d[tid];
  __syncthreads();
  const double alpha = ctl->alpha;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  double acc = 0.0;
  if (i < cfg.n) {
    double vi[KB];
#pragma unroll
    for (int l = 0; l < KB; ++l) vi[l] = (l < r) ? (double)Qw[i * KB + l] * sd[l] : 0.0;
    for (int64_t j = lane; j < cfg.n; j += 64) {
      double x = (j == i) ? alpha : 0.0;
#pragma unroll
      for (int l = 0; l < KB; ++l)
        if (l < r) x += vi[l] * (double)Qw[j * KB + l];
      const double dij = (double)D[i * cfg.ld + j];
      if (cfg.kind == LINEAR_DENSE) acc += dij * x;
      else acc += 0.5 * (x - dij) * (x - dij);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) sred[wave] = acc;
  __syncthreads();
  if (tid == 0) { mine[0] = sred[0] + sred[1] + sred[2] + sred[3]; mine[1] = 0.0; }
  __syncthreads();
  if (tree_reduce<256>(red, mine, mine)) {
    if (tid == 0) { ctl->f = mine[0]; ctl->fvalid = 1; }
  }
}

// objective at X_t, CSR kinds (LINEAR: sum_Omega C_ij X_ij; MASKED: 1/2 sum_Omega (X_ij - M_ij)^2)
template <typename T, int KB>
__global__ __launch_bounds__(256) void k_objective_csr(Cfg cfg, Ctl* __restrict__ ctl, const int* __restrict__ rp,
                                                       const int* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ Qw, Red red) {
  __shared__ double sd[KMAX];
  __shared__ double sred[4];
  __shared__ double mine[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = cfg.r;
  if (tid < KMAX) sd[tid] = ctl->d[tid];
  __syncthreads();
  const double alpha = ctl->alpha;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  double acc = 0.0;
  if (i < cfg.n) {
    double vi[KB];
#pragma unroll
    for (int l = 0; l < KB; ++l) vi[l] = (l < r) ? (double)Qw[i * KB + l] * sd[l] : 0.0;
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) {
      const int64_t j = col[e];
      double x = (j == i) ? alpha : 0.0;
#pragma unroll
      for (int l = 0; l < KB; ++l)
        if (l < r) x += vi[l] * (double)Qw[j * KB + l];
      const double v = (double)val[e];
      if (cfg.kind == LINEAR_CSR) acc += v * x;
      else acc += 0.5 * (x - v) * (x - v);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) sred[wave] = acc;
  __syncthreads();
  if (tid == 0) { mine[0] = sred[0] + sred[1] + sred[2] + sred[3]; mine[1] = 0.0; }
  __syncthreads();
  if (tree_reduce<256>(red, mine, mine)) {
    if (tid == 0) { ctl->f = mine[0]; ctl->fvalid = 1; }
  }
}

// ---------------------------------------------------------------------------
// y = Op x for the data operator (dense C/M or the CSR values), FP64 result.
// Used once per context by the Lanczos estimate of the operator's extreme
// eigenvalues.  One wave per row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_matvec(Cfg cfg, const T* __restrict__ D, const int* __restrict__ rp,
                                                const int* __restrict__ col, const T* __restrict__ val,
                                                const T* __restrict__ x, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= cfg.n) return;
  double acc = 0.0;
  if (cfg.kind == LINEAR_DENSE || cfg.kind == DENOISE_DENSE) {
    for (int64_t j = lane; j < cfg.n; j += 64) acc += (double)D[i * cfg.ld + j] * (double)x[j];
  } else {
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) acc += (double)val[e] * (double)x[col[e]];
  }
  acc = wave_sum(acc);
  if (lane == 0) y[i] = acc;
}

// CSR structure check: 0 = rp[0] <= rp[i] <= rp[i+1] <= rp[n] = nnz and every
// column index in [0, n).  Row ranges are validated before col is read.
__global__ __launch_bounds__(256) void k_check_csr(const int* __restrict__ rp, const int* __restrict__ col,
                                                   int64_t n, int64_t nnz, int* __restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t a = rp[i], b = rp[i + 1];
    int bad = 0;
    if (i == 0 && a != 0) bad = 1;
    if (i == n - 1 && b != nnz) bad = 1;
    if (a < 0 || b < a || b > nnz) bad = 1;
    if (!bad)
      for (int64_t e = a; e < b; ++e) {
        const int c = col[e];
        if (c < 0 || c >= n) { bad = 1; break; }
      }
    if (bad) atomicOr(err, 1);
  }
}

// ---------------------------------------------------------------------------
// data norm: sqrt(sum of squares) of a strided matrix (rows x cols, ld) or a
// vector (rows = 1); grid-stride, FP64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T* __restrict__ x, int64_t rows, int64_t cols, int64_t ld,
                                               Ctl* __restrict__ ctl, Red red) {
  __shared__ double sred[4];
  __shared__ double mine[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc = 0.0;
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e % cols;
    const double v = (double)x[i * ld + j];
    acc += v * v;
  }
  acc = wave_sum(acc);
  if (lane == 0) sred[wave] = acc;
  __syncthreads();
  if (tid == 0) { mine[0] = sred[0] + sred[1] + sred[2] + sred[3]; mine[1] = 0.0; }
  __syncthreads();
  if (tree_reduce<256>(red, mine, mine)) {
    if (tid == 0) ctl->data_norm = sqrt(mine[0]);
  }
}

}  // namespace meg
