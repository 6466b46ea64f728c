// HIP kernels of the low-rank MEG step (gfx950, wave64).
//
// One step t (Algorithm 2, Section 3) runs inside ONE persistent, cooperatively
// launched kernel (k_step), phases separated by grid barriers:
//   grad   : masked objective: gradient values on Omega at X_t, f(X_t) and the
//            norms that set the solver's shift (other objectives: shift only)
//   sweep s: apply   Zout = Yhat (Zin W) for the implicit orthonormal basis
//                    Q = Zin W, Yhat = V diag(ceff) V^T + opscale*Op + sdiag*I,
//                    with FP64 Gram partials Zin^T Zout, Zout^T Zout, V^T Zout
//            barrier the partials are summed along the arrival tree
//            small   Cholesky QR (sweep 1) or Rayleigh-Ritz + Cholesky QR in
//                    FP64, one wavefront of the last workgroup to arrive;
//                    stops the sweep loop when the Ritz residuals meet the
//                    tolerance
//   final  : Qw <- Zsrc Wfin (Ritz basis = next warm start; its first r
//            columns are V_{t+1}) and its Gram, whose Cholesky factor
//            orthonormalises the first sweep of step t+1
// Cross-workgroup communication happens only at the barriers, so no
// workgroup writes back or invalidates the L2 while others stream through it.
#pragma once
#include "meg_device.hpp"
#include "meg_small.hpp"

namespace meg {

enum OpKind : int { OP_CSR = 0, OP_DENSE = 1 };

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

// Scratch doubles the small solves need (they reuse the apply's LDS).
template <int KB>
constexpr int small_scratch() { return 5 * KB * (KB + 1) + 8 * KB; }

// Rows per wave of the dense apply: keep RPW * KB accumulators per lane modest.
template <typename T, int KB>
constexpr int dense_rpw() { return (KB * (int)sizeof(T) <= 64) ? 4 : ((KB * (int)sizeof(T) <= 128) ? 2 : 1); }

template <typename T, int KB, int OPK, int NT>
struct StepShape {
  static constexpr int WAVES = NT / 64;
  static constexpr int RPW = (OPK == OP_CSR) ? 1 : dense_rpw<T, KB>();
  static constexpr int ROWS = WAVES * RPW;  // rows per apply block
  static constexpr int FROWS = 2 * WAVES;   // rows per finalize block
};

template <typename T, int KB, int ROWS>
struct ApplySmem {
  static constexpr int LD = KB + 1;
  // typed section (in units of T)
  static constexpr int T_W = 0;                  // KB x LD
  static constexpr int T_P = T_W + KB * LD;      // KB x KB (r rows used)
  static constexpr int T_CE = T_P + KB * KB;     // KB
  static constexpr int T_ZIN = T_CE + KB;        // ROWS x KB
  static constexpr int T_V = T_ZIN + ROWS * KB;  // ROWS x KB
  static constexpr int T_U = T_V + ROWS * KB;    // ROWS x KB
  static constexpr int T_ZO = T_U + ROWS * KB;   // ROWS x KB
  static constexpr int T_END = T_ZO + ROWS * KB;
  static constexpr int TYPED_DOUBLES = (T_END * (int)sizeof(T) + 7) / 8;
  static constexpr int PLEN = 3 * KB * KB;       // Gram accumulator (FP64)
  static constexpr int SMALL = small_scratch<KB>();
  static constexpr int BODY = TYPED_DOUBLES > SMALL ? TYPED_DOUBLES : SMALL;
  static constexpr int TOTAL = PLEN + BODY;
};

// Operand pointers of the objective.
template <typename T>
struct Data {
  const int* rp;
  const int* col;
  const T* val;  // CSR values (M_Omega or C)
  const T* D;    // dense C or M
};

// ---------------------------------------------------------------------------
// step scalars for objectives without a gradient pass (single thread)
// ---------------------------------------------------------------------------
__device__ inline void prep_scalars(const Cfg& cfg, Ctl* ctl, int lane) {
  double gmax;
  if (cfg.kind == DENOISE_DENSE) {
    // lambda_max(X - M) <= lambda_max(X) - lambda_min(M), lambda_max(X) = alpha + max(0, max d)
    const double dmax = wave_max(lane < cfg.r ? fmax(ctl->d[lane], 0.0) : 0.0);
    gmax = ctl->alpha + dmax - ctl->op_lmin;
  } else {
    gmax = ctl->op_lmax;  // G = C
  }
  setup_step(cfg, ctl, gmax, lane);
}

// Sum of the 2-value per-workgroup partials of the gradient phase, in a fixed
// order (one wavefront).
__device__ inline void sum_pairs(const double* part, int P, int lane, double* s0, double* s1) {
  double a = 0.0, b = 0.0;
  for (int p0 = 0; p0 < P; p0 += 64 * 8) {  // P <= 1024: at most 2 rounds of 8 loads in flight
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int p = p0 + lane + 64 * u;
      va[u] = (p < P) ? part[2 * p] : 0.0;
      vb[u] = (p < P) ? part[2 * p + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a += va[u];
      b += vb[u];
    }
  }
  *s0 = wave_sum(a);
  *s1 = wave_sum(b);
}

// ---------------------------------------------------------------------------
// gradient phase (masked CSR): g_e = X_ij - M_ij on Omega, with
// X_ij = alpha [i == j] + sum_l V_il d_l V_jl; per-workgroup partials
// (sum g^2, sum X_ij^2) -> part[wg * 2].  One wave per row, grid-stride.
// ---------------------------------------------------------------------------
template <typename T, int KB, int NT>
__device__ __noinline__ void grad_phase(const Cfg& cfg, const Ctl* ctl, const Data<T>& dat, const T* __restrict__ Qw,
                           T* __restrict__ g, double* part, double* lds) {
  constexpr int WAVES = NT / 64;
  T* sd = reinterpret_cast<T*>(lds);      // KMAX
  double* sred = lds + KMAX;               // 2 * WAVES
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = cfg.r;
  if (tid < KMAX) sd[tid] = (T)ctl->d[tid];
  const T alpha = (T)ctl->alpha;
  __syncthreads();
  constexpr int VN = V16<T>::N;
  constexpr int U = 2;  // nonzeros per lane per iteration, loads issued together
  double acc = 0.0, accx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * WAVES + wave; i < cfg.n; i += (int64_t)gridDim.x * WAVES) {
    // vi_l = V_il d_l; d_l = 0 for l >= r, so whole k-wide rows can be used
    T vi[KB];
#pragma unroll
    for (int l = 0; l < KB; ++l) vi[l] = (l < r) ? Qw[i * KB + l] * sd[l] : (T)0;
    const int e0 = dat.rp[i], e1 = dat.rp[i + 1];
    for (int e = e0 + lane; e < e1; e += 64 * U) {
      int jj[U];
      T mv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int eu = e + 64 * u;
        const bool ok = eu < e1;
        jj[u] = ok ? dat.col[eu] : (int)i;
        mv[u] = ok ? dat.val[eu] : (T)0;
      }
      T vj[U][KB];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < KB / VN; ++c) vload<T>(Qw + (int64_t)jj[u] * KB + c * VN, &vj[u][c * VN]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int eu = e + 64 * u;
        T x = (jj[u] == i) ? alpha : (T)0;
#pragma unroll
        for (int l = 0; l < KB; ++l) x += vi[l] * vj[u][l];
        if (eu < e1) {
          const T gvv = x - mv[u];
          g[eu] = gvv;
          acc += (double)gvv * (double)gvv;
          accx += (double)x * (double)x;
        }
      }
    }
  }
  acc = wave_sum(acc);
  accx = wave_sum(accx);
  if (lane == 0) {
    sred[wave] = acc;
    sred[WAVES + wave] = accx;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < WAVES; ++w) { a += sred[w]; b += sred[WAVES + w]; }
    part[(size_t)blockIdx.x * 2] = a;
    part[(size_t)blockIdx.x * 2 + 1] = b;
  }
}

// ---------------------------------------------------------------------------
// apply phase: all row blocks of this workgroup, Gram partials -> part[wg]
// ---------------------------------------------------------------------------
template <typename T, int KB, int OPK, int NT>
__device__ void apply_phase(const Cfg& cfg, const Ctl* ctl, const Data<T>& dat, const T* __restrict__ gv,
                            const T* __restrict__ Qw, const T* __restrict__ Zin, T* __restrict__ Zout,
                            double* part, double* smem) {
  using SH = StepShape<T, KB, OPK, NT>;
  constexpr int ROWS = SH::ROWS, RPW = SH::RPW;
  using SM = ApplySmem<T, KB, ROWS>;
  constexpr int LD = SM::LD;
  constexpr int VN = V16<T>::N;
  T* tb = reinterpret_cast<T*>(smem + SM::PLEN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = cfg.r;
  const int64_t n = cfg.n;
  // per-sweep coefficients
  for (int e = tid; e < KB * KB; e += NT) {
    tb[SM::T_W + (e / KB) * LD + (e % KB)] = (T)ctl->W[e];
    tb[SM::T_P + e] = (e / KB < r) ? (T)ctl->Pin[e] : (T)0;
  }
  if (tid < KB) tb[SM::T_CE + tid] = (T)ctl->ceff[tid];
  for (int e = tid; e < SM::PLEN; e += NT) smem[e] = 0.0;
  const T opscale = (T)ctl->opscale, sdiag = (T)ctl->sdiag;
  const int64_t nblk = (n + ROWS - 1) / ROWS;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t row0 = blk * ROWS;
    __syncthreads();  // previous block's LDS reads are done
    for (int e = tid; e < ROWS * KB; e += NT) {
      const int rr = e / KB, cc = e % KB;
      const int64_t i = row0 + rr;
      const bool ok = i < n;
      tb[SM::T_ZIN + e] = ok ? Zin[i * KB + cc] : (T)0;
      tb[SM::T_V + e] = (ok && cc < r) ? Qw[i * KB + cc] : (T)0;
    }
    if constexpr (OPK == OP_CSR) {
      // one row per wave; a row's nonzeros are split over lane groups of LPN
      // lanes, each lane owning a 16-byte chunk of the gathered Zin row
      constexpr int LPN = KB / VN;
      constexpr int NPI = 64 / LPN;
      const int sub = lane % LPN, grp = lane / LPN;
      const int64_t i = row0 + wave;
      T acc[VN];
#pragma unroll
      for (int v = 0; v < VN; ++v) acc[v] = 0;
      if (i < n) {
        // U nonzeros per lane group per iteration: all index/value loads,
        // then all row gathers, are issued before the first use
        constexpr int U = 4;
        const int e0 = dat.rp[i], e1 = dat.rp[i + 1];
        for (int e = e0 + grp; e < e1; e += NPI * U) {
          int jj[U];
          T ww[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int eu = e + u * NPI;
            const bool ok = eu < e1;
            jj[u] = ok ? dat.col[eu] : (int)i;  // in-range row, weight 0
            ww[u] = ok ? gv[eu] : (T)0;
          }
          T z[U][VN];
#pragma unroll
          for (int u = 0; u < U; ++u) vload<T>(Zin + (int64_t)jj[u] * KB + sub * VN, z[u]);
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < VN; ++v) acc[v] += ww[u] * z[u][v];
        }
      }
#pragma unroll
      for (int o = LPN; o < 64; o <<= 1)
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] += __shfl_xor(acc[v], o, 64);
      if (grp == 0) {
#pragma unroll
        for (int v = 0; v < VN; ++v) tb[SM::T_U + wave * KB + sub * VN + v] = acc[v];
      }
    } else {
      // dense: each wave owns RPW rows; column chunks of 64 with the matching
      // 64 rows of Zin staged in LDS once for all rows of the block
      T* zc = tb + SM::T_END;  // 64 x LD
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
          zc[jj * LD + c] = (j < n) ? Zin[j * KB + c] : (T)0;
        }
        __syncthreads();
        const int64_t j = j0 + lane;
        T dv[RPW];
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
          const int64_t i = row0 + wave * RPW + q;
          dv[q] = (i < n && j < n) ? dat.D[i * cfg.ld + j] : (T)0;
        }
#pragma unroll
        for (int c = 0; c < KB; ++c) {
          const T z = zc[lane * LD + c];
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
    }
    __syncthreads();
    // u = opscale*(Op Zin)_i + V_i diag(ceff) Pin + sdiag Zin_i   (Zin basis)
    for (int e = tid; e < ROWS * KB; e += NT) {
      const int rr = e / KB, a = e % KB;
      T u = opscale * tb[SM::T_U + e] + sdiag * tb[SM::T_ZIN + e];
      for (int l = 0; l < r; ++l) u += tb[SM::T_V + rr * KB + l] * tb[SM::T_CE + l] * tb[SM::T_P + l * KB + a];
      tb[SM::T_ZO + e] = u;
    }
    __syncthreads();
    // z = u W (rows beyond n are zero)
    for (int e = tid; e < ROWS * KB; e += NT) {
      const int rr = e / KB, b = e % KB;
      T z = 0;
#pragma unroll 8
      for (int a = 0; a < KB; ++a) z += tb[SM::T_ZO + rr * KB + a] * tb[SM::T_W + a * LD + b];
      const int64_t i = row0 + rr;
      if (i < n) Zout[i * KB + b] = z; else z = 0;
      tb[SM::T_U + e] = z;
    }
    __syncthreads();
    // FP64 Gram partials (products of working-precision values are exact)
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
      smem[e] += c;
      smem[KB * KB + e] += gg;
      smem[2 * KB * KB + e] += p;
    }
  }
  __syncthreads();
  double* dst = part + (size_t)blockIdx.x * SM::PLEN;
  for (int e = tid; e < SM::PLEN; e += NT) dst[e] = smem[e];
}

// ---------------------------------------------------------------------------
// finalize phase: Qw <- Zsrc Wfin (row-local, in place when Zsrc == Qw) and
// the Gram partial of the new Qw -> part[wg] (KB x KB)
// mode 0: end of a step; mode 1: fresh basis (Wfin = I)
// ---------------------------------------------------------------------------
template <typename T, int KB, int FROWS, int NT>
__device__ __noinline__ void finalize_phase(const Cfg& cfg, const Ctl* ctl, T* __restrict__ Qw, const T* Zs, int mode,
                               double* part, double* smem) {
  constexpr int LD = KB + 1;
  double* acc = smem;                                   // KB * KB
  T* sWf = reinterpret_cast<T*>(smem + KB * KB);        // KB x LD
  T* rin = sWf + KB * LD;                               // FROWS x KB
  T* rout = rin + FROWS * KB;                           // FROWS x KB
  const int tid = threadIdx.x;
  const int64_t n = cfg.n;
  for (int e = tid; e < KB * KB; e += NT) {
    sWf[(e / KB) * LD + (e % KB)] = (mode == 0) ? (T)ctl->Wfin[e] : (T)((e / KB) == (e % KB));
    acc[e] = 0.0;
  }
  const int64_t nblk = (n + FROWS - 1) / FROWS;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t row0 = blk * FROWS;
    __syncthreads();
    for (int e = tid; e < FROWS * KB; e += NT) {
      const int64_t i = row0 + e / KB;
      rin[e] = (i < n) ? Zs[i * KB + e % KB] : (T)0;
    }
    __syncthreads();
    for (int e = tid; e < FROWS * KB; e += NT) {
      const int rr = e / KB, b = e % KB;
      T z = 0;
#pragma unroll 8
      for (int a = 0; a < KB; ++a) z += rin[rr * KB + a] * sWf[a * LD + b];
      const int64_t i = row0 + rr;
      if (i < n) Qw[i * KB + b] = z; else z = 0;
      rout[e] = z;
    }
    __syncthreads();
    for (int e = tid; e < KB * KB; e += NT) {
      const int a = e / KB, b = e % KB;
      double s = 0.0;
#pragma unroll 4
      for (int rr = 0; rr < FROWS; ++rr) s += (double)rout[rr * KB + a] * (double)rout[rr * KB + b];
      acc[e] += s;
    }
  }
  __syncthreads();
  double* dst = part + (size_t)blockIdx.x * KB * KB;
  for (int e = tid; e < KB * KB; e += NT) dst[e] = acc[e];
}

template <typename T>
__device__ __forceinline__ T* zbuf(T* Qw, T* Za, T* Zb, int i) {
  return i == 0 ? Qw : (i == 1 ? Za : Zb);
}

__device__ __forceinline__ int ldi(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void stamp(const Bufs& b, int slot) {
  if (b.ts && threadIdx.x == 0) b.ts[slot] = wall_clock64();
}

// ---------------------------------------------------------------------------
// persistent step kernel: `nsteps` iterations of Algorithm 2, or (mode 1) a
// fresh-basis setup only.  Launched cooperatively (all workgroups resident).
// Grid barriers per iteration: one after the gradient, one per sweep (its
// Gram partials are summed on the way through the barrier) and one after the
// basis update.
// ---------------------------------------------------------------------------
template <typename T, int KB, int OPK, int NT>
__global__ __launch_bounds__(NT) void k_step(Cfg cfg, Ctl* __restrict__ ctl, Data<T> dat, T* __restrict__ Qw,
                                             T* __restrict__ Za, T* __restrict__ Zb, T* __restrict__ g, Bufs b,
                                             int nsteps) {
  using SH = StepShape<T, KB, OPK, NT>;
  using SM = ApplySmem<T, KB, SH::ROWS>;
  constexpr int DENSE_STAGE = (OPK == OP_DENSE) ? (64 * (KB + 1) * (int)sizeof(T) + 7) / 8 : 0;
  __shared__ double smem[SM::TOTAL + DENSE_STAGE];
  const int tid = threadIdx.x;
  const int P = gridDim.x;

  for (int st = 0; st < nsteps; ++st) {
    if (ldi(&ctl->stop) | ldi(&ctl->status)) break;
    if (blockIdx.x == 0) stamp(b, 0);
    // ---- gradient at X_t / step scalars
    if (cfg.kind == MASKED_CSR) grad_phase<T, KB, NT>(cfg, ctl, dat, Qw, g, b.part, smem);
    if (!grid_sync<NT>(b, 0, [&] {
          if (tid < 64) {
            if (cfg.kind == MASKED_CSR) {
              double s0, s1;
              sum_pairs(b.part, P, tid, &s0, &s1);
              if (tid == 0) {
                ctl->f = 0.5 * s0;
                ctl->fvalid = 1;
              }
              // lambda_max(P(X) - P(M)) <= ||P(X)||_F - lambda_min(P(M)),  P = P_Omega
              setup_step(cfg, ctl, sqrt(s1) - ctl->op_lmin, tid);
            } else {
              prep_scalars(cfg, ctl, tid);
            }
          }
          stamp(b, 1);
        }))
      return;
    // ---- block subspace sweeps with Rayleigh-Ritz
    const T* gvals = (cfg.kind == MASKED_CSR) ? g : dat.val;
    for (int s = 1; s <= cfg.max_inner; ++s) {
      const int in = (s == 1) ? 0 : ((s % 2 == 0) ? 1 : 2);
      const int out = (s == 1) ? 1 : ((s % 2 == 0) ? 2 : 1);
      apply_phase<T, KB, OPK, NT>(cfg, ctl, dat, gvals, Qw, zbuf(Qw, Za, Zb, in), zbuf(Qw, Za, Zb, out), b.part,
                                  smem);
      if (!grid_sync<NT>(b, SM::PLEN, [&] {
            stamp(b, 2 * s);
            if (tid < 64) small_sweep<KB>(cfg, ctl, b.sums, smem, s, in, tid);
            if (tid == 0) ctl->applies_done = ctl->applies_done + 1;
            stamp(b, 2 * s + 1);
          }))
        return;
      if (ldi(&ctl->done) | ldi(&ctl->status)) break;
    }
    if (ldi(&ctl->status)) break;
    // ---- next warm-start basis and iterate
    const T* Zs = zbuf(Qw, Za, Zb, ldi(&ctl->src));
    finalize_phase<T, KB, SH::FROWS, NT>(cfg, ctl, Qw, Zs, 0, b.part, smem);
    if (!grid_sync<NT>(b, KB * KB, [&] {
          stamp(b, 2 * cfg.max_inner + 2);
          if (tid < 64) basis_setup<KB>(cfg, ctl, b.sums, smem, tid);
          if (tid == 0) {
            ctl->t = ctl->t + 1;
            ctl->iters_done = ctl->iters_done + 1;
            ctl->fvalid = 0;
          }
          stamp(b, 2 * cfg.max_inner + 3);
        }))
      return;
  }
}

// Orthonormalising transform of a freshly uploaded basis Qw (cooperative
// launch with the step kernel's grid): Gram of Qw, then the transform that
// makes Qw W an orthonormal basis for the first sweep of the next step.
template <typename T, int KB, int OPK, int NT>
__global__ __launch_bounds__(NT) void k_basis(Cfg cfg, Ctl* __restrict__ ctl, T* __restrict__ Qw, Bufs b) {
  using SH = StepShape<T, KB, OPK, NT>;
  using SM = ApplySmem<T, KB, SH::ROWS>;
  __shared__ double smem[SM::TOTAL];
  const int tid = threadIdx.x;
  finalize_phase<T, KB, SH::FROWS, NT>(cfg, ctl, Qw, Qw, 1, b.part, smem);
  grid_sync<NT>(b, KB * KB, [&] {
    if (tid < 64) basis_setup<KB>(cfg, ctl, b.sums, smem, tid);
  });
}

// ---------------------------------------------------------------------------
// auxiliary kernels (ordinary launches; per-workgroup partials, then k_finish)
// ---------------------------------------------------------------------------
// objective at X_t, dense kinds: LINEAR sum C_ij X_ij, DENOISE 1/2 sum (X_ij - M_ij)^2
// X_ij = alpha [i == j] + sum_l V_il d_l V_jl, accumulated in FP64; one wave per row
template <typename T, int KB>
__global__ __launch_bounds__(256) void k_objective_dense(Cfg cfg, const Ctl* __restrict__ ctl,
                                                         const T* __restrict__ D, const T* __restrict__ Qw,
                                                         double* __restrict__ part) {
  __shared__ double sd[KMAX];
  __shared__ double sred[4];
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
  if (tid == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// objective at X_t, CSR kinds (LINEAR: sum_Omega C_ij X_ij; MASKED: 1/2 sum_Omega (X_ij - M_ij)^2)
template <typename T, int KB>
__global__ __launch_bounds__(256) void k_objective_csr(Cfg cfg, const Ctl* __restrict__ ctl, const int* __restrict__ rp,
                                                       const int* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ Qw, double* __restrict__ part) {
  __shared__ double sd[KMAX];
  __shared__ double sred[4];
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
  if (tid == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// sum of squares of a strided matrix (rows x cols, ld) or a vector (rows = 1)
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T* __restrict__ x, int64_t rows, int64_t cols, int64_t ld,
                                               double* __restrict__ part) {
  __shared__ double sred[4];
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
  if (tid == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// Sum nwg partials in a fixed order and store: what = 0 -> f (objective),
// 1 -> data_norm = sqrt(sum).  One workgroup.
__global__ __launch_bounds__(256) void k_finish(Ctl* __restrict__ ctl, const double* __restrict__ part, int nwg,
                                                int what) {
  __shared__ double s[256];
  double a = 0.0;
  for (int w = threadIdx.x; w < nwg; w += 256) a += part[w];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (what == 0) {
      ctl->f = s[0];
      ctl->fvalid = 1;
    } else {
      ctl->data_norm = sqrt(s[0]);
    }
  }
}

// y = Op x for the data operator (dense C/M or the CSR values), FP64 result.
// Used once per context by the Lanczos estimate of the operator's extreme
// eigenvalues.  One wave per row.
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

}  // namespace meg
