// HIP kernels of the low-rank MEG step (gfx950, wave64).
//
// One step t (Algorithm 2, Section 3) runs inside ONE persistent, cooperatively
// launched kernel (k_step), phases separated by grid barriers:
//   sweep s: apply   Zout = Yhat (Zin W) for the implicit orthonormal basis
//                    Q = Zin W, Yhat = V diag(ceff) V^T + opscale*Op + sdiag*I,
//                    with FP64 Gram partials Zin^T Zout, Zout^T Zout, V^T Zout;
//                    in sweep 1 of the masked objective the gradient values on
//                    Omega at X_t (and f(X_t)) are formed from the same gathers
//            barrier the partials are summed along the arrival tree
//            small   Cholesky QR (sweep 1) or Rayleigh-Ritz + Cholesky QR in
//                    FP64, one wavefront of the last workgroup to arrive;
//                    stops the sweep loop when the Ritz residuals meet the
//                    tolerance
// The step ends in the small solve of its last sweep: the Ritz basis of that
// sweep, Zin (W S), is the next warm start, kept implicit as (B, Wb) = (Zin,
// W S) so no pass over the n x k block is needed; the shift and
// coefficients of step t+1 follow from the new factored iterate.
// Cross-workgroup communication happens only at the barriers, so no
// workgroup writes back or invalidates the L2 while others stream through it.
#pragma once
#include <type_traits>

#include "meg_device.hpp"
#include "meg_small.hpp"

namespace meg {

// Operator families of the apply: sparse CSR, dense in the state's type,
// dense given as two bf16 planes hi + lo and applied on the matrix cores, and
// the factored minibatch gradient A_B^T diag(w / L) A_B.
enum OpKind : int { OP_CSR = 0, OP_DENSE = 1, OP_DENSE_X3 = 2, OP_FACTOR = 3 };

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

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of
// a group receives its group's sum.  Exchanges within a quad use DPP quad
// permutes (xor 1: [1,0,3,2], xor 2: [2,3,0,1]); wider ones use shuffles.
__device__ __forceinline__ float dpp_xor(float v, int m) {
  const int x = __float_as_int(v);
  return __int_as_float(m == 1 ? __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true)
                               : __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ double dpp_xor(double v, int m) {
  const long long b = __double_as_longlong(v);
  int lo = (int)b, hi = (int)(b >> 32);
  if (m == 1) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, true);
    hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, true);
  } else {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, true);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, true);
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if constexpr (G >= 2) v += dpp_xor(v, 1);
  if constexpr (G >= 4) v += dpp_xor(v, 2);
#pragma unroll
  for (int o = 4; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Scratch doubles the small solves need (they reuse the apply's LDS).
template <int KB>
constexpr int small_scratch() { return 5 * KB * (KB + 1) + 12 * KB; }

// Rows per wave of the dense apply: keep RPW * KB accumulators per lane modest.
template <typename T, int KB>
constexpr int dense_rpw() { return (KB * (int)sizeof(T) <= 64) ? 4 : ((KB * (int)sizeof(T) <= 128) ? 2 : 1); }

template <typename T, int KB, int OPK, int NT>
struct StepShape {
  static constexpr int WAVES = NT / 64;
  // rows per wave: CSR rows are gathered concurrently (more loads in flight);
  // the matrix-core form works on 64-row blocks (two 32-row MFMA tiles)
  static constexpr int RPW = (OPK == OP_CSR) ? 2
                             : (OPK == OP_DENSE_X3 ? 64 / WAVES : (OPK == OP_FACTOR ? 32 / WAVES : dense_rpw<T, KB>()));
  static constexpr int ROWS = WAVES * RPW;  // rows per apply block
  static constexpr int GROWS = 2 * WAVES;   // rows per block of the basis Gram
  static constexpr int GWROWS = (OPK == OP_CSR) ? ROWS : 0;  // fused-gradient scratch rows
};

template <typename T, int KB, int ROWS, int GWROWS = ROWS>
struct ApplySmem {
  static constexpr int LD = KB + 1;
  // typed section (in units of T)
  static constexpr int T_W = 0;                   // KB x LD   sweep transform W
  static constexpr int T_WB = T_W + KB * LD;      // KB x LD   basis transform Wb
  static constexpr int T_PW = T_WB + KB * LD;     // KB x KB   V^T Q (r rows used)
  static constexpr int T_CE = T_PW + KB * KB;     // KB
  static constexpr int T_ZIN = T_CE + KB;         // ROWS x KB
  static constexpr int T_B = T_ZIN + ROWS * KB;   // ROWS x KB basis rows
  static constexpr int T_V = T_B + ROWS * KB;     // ROWS x KB V rows (zero beyond r)
  static constexpr int T_U = T_V + ROWS * KB;     // ROWS x KB
  static constexpr int T_ZO = T_U + ROWS * KB;    // ROWS x KB
  static constexpr int T_GW = T_ZO + ROWS * KB;   // GWROWS x 3 x KB, fused gradient
  static constexpr int T_END = T_GW + 3 * GWROWS * KB;
  // explicit residuals of the previous Rayleigh-Ritz sweep (FP64 state only);
  // its input rows go to the T_B rows once those are used up
  static constexpr int XR = sizeof(T) == 8 ? 1 : 0;
  static constexpr int TYPED_DOUBLES = (T_END * (int)sizeof(T) + 7) / 8;
  static constexpr int PLEN = 3 * KB * KB;       // Gram accumulators (FP64): Zin^T Zout, G, P
  // longest per-workgroup partial record (PartRec; its length depends on r)
  static constexpr int PSTRIDE = PartRec<KB>::len(KB - 1, XR != 0);
  static constexpr int ACC = PLEN + XR * KB;     // accumulators: Gram, residual column sums
  static constexpr int SMALL = small_scratch<KB>();
  static constexpr int BODY = TYPED_DOUBLES > SMALL ? TYPED_DOUBLES : SMALL;
  // the reduced record, summed into LDS by the barrier's last arrival for
  // the small solve (after its scratch)
  static constexpr int SUMS = SMALL;
  static constexpr int TOTAL = ACC + BODY > SUMS + PSTRIDE ? ACC + BODY : SUMS + PSTRIDE;
};

// Operand pointers of the objective.
template <typename T>
struct Data {
  const int* rp;
  const int* col;
  const T* val;          // CSR values (M_Omega or C)
  const T* D;            // dense C or M
  const uint16_t* Dhi;   // dense, as bf16 planes hi + lo (matrix-core form)
  const uint16_t* Dlo;
  // factored minibatch gradient (quadratic measurements)
  const T* A;            // pool, measurement i = row i (stride lda)
  const T* bq;           // measured values b[m]
  const int* bidx;       // minibatch indices (batch_steps x L; the step's row in k_step)
  T* qy;                 // L x KB: y_i = (w_i / L) a_i^T Zin
  T* qk;                 // L x L: minibatch Gram matrix A_B A_B^T (first sweep)
  double* qw;            // L: residuals w_i = a_i^T X_t a_i - b_i
  double* qn;            // L: ||a_i||^2
};

// This workgroup's slice of the CSR data in LDS (see cache_layout): row
// starts as cache positions, column indices, values, and the values the
// later sweeps apply (gradient values for the masked objective, else the
// values themselves).
template <typename T>
struct CsrCache {
  lds<int>* rloc;
  lds<int>* col;
  lds<T>* val;
  lds<T>* g;
  lds<T>* gv;
};

// Fill the cache at the start of a launch: the row blocks tm.wg,
// tm.wg + tm.nwg, ... in order, their entries contiguous.  Rows past
// n are empty.  All threads call it; ends with a workgroup barrier.
template <typename T, int ROWS, int NT>
__device__ void load_csr_cache(const Cfg& cfg, const Data<T>& dat, const CsrCache<T>& cc, Team tm) {
  const int tid = threadIdx.x;
  const int64_t n = cfg.n;
  const int64_t nblk = (n + ROWS - 1) / ROWS;
  int off = 0;  // cache position of the current block's first entry
  int jb = 0;
  for (int64_t blk = tm.wg; blk < nblk; blk += tm.nwg, ++jb) {
    const int64_t row0 = blk * ROWS;
    const int64_t rend = (row0 + ROWS < n) ? row0 + ROWS : n;
    const int base = dat.rp[row0];
    const int cnt = dat.rp[rend] - base;
    for (int t = tid; t <= ROWS; t += NT) {
      const int64_t row = (row0 + t < rend) ? row0 + t : rend;
      cc.rloc[jb * (ROWS + 1) + t] = off + (dat.rp[row] - base);
    }
    for (int e = tid; e < cnt; e += NT) {
      cc.col[off + e] = dat.col[base + e];
      cc.val[off + e] = dat.val[base + e];
    }
    off += cnt;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// step scalars of the NEXT iteration t, set before it starts (one
// wavefront).  gmax >= lambda_max(grad f(X_t)):
//   linear   G = C:               lambda_max(C)
//   denoise  G = X - M:           lambda_max(X) - lambda_min(M), lambda_max(X) = alpha + max(0, max d)
//   masked   G = P(X) - P(M):     ||P(X_t)||_2 - lambda_min(P(M))   (P = P_Omega), with
//            ||P(X_t)||_2 <= ||P(X_{t-1})||_F + ||X_t - X_{t-1}||_F  (both known
//            from the previous step), or ||P(X_t)||_2 <= ||X_t||_F with
//            ||X_t||_F^2 = (n - r) alpha^2 + sum_l (alpha + d_l)^2 after a new start
// so the shift needs no pass over the data and the gradient can be formed
// inside the first sweep.  A caller-supplied G_t (external gradient) is a
// linear operator for the step: lambda_max is its Gershgorin bound, from one
// pass over G_t before the step (k_gersh_dense / k_gersh_csr).
// ---------------------------------------------------------------------------
__device__ inline void step_scalars(const Cfg& cfg, gbl<Ctl>* ctl, int lane) {
  // the minibatch gradient's bound is known only inside sweep 1 (factor_shift)
  if (cfg.kind == QUADMEAS) return;
  const bool act = lane < cfg.r;
  const double alpha = ctl->alpha, dl = act ? ctl->d[lane] : 0.0, cl = act ? ctl->c[lane] : 0.0;
  const double gmax =
      grad_bound(cfg, alpha, dl, ctl->op_lmin, ctl->op_lmax, ctl->pxvalid, ctl->pxnorm, ctl->dxnorm, lane);
  setup_step_v(cfg, ctl, gmax, alpha, dl, cl, ctl->mu_1, ctl->mu_k, ctl->mu_valid, lane);
}

// ---------------------------------------------------------------------------
// Dense product on the matrix cores, three bf16 passes with FP32 accumulation:
//   out = M[row0:row0+64, :] Zin,   M = Mhi + Mlo (two bf16 planes),
//   Zin = Zhi + Zlo split in the same way as it is staged,
//   M Zin ~ Mhi Zhi + Mhi Zlo + Mlo Zhi  (the Mlo Zlo term is below 2^-16).
// 512 threads: wave w owns the 32-row tile w % 2 and the K quarter w / 2 of
// every K chunk of 256.  K is traversed in an order of our choosing (the sum
// does not depend on it): lane (i, h) of a wave reads 64 contiguous bytes of
// row i of each plane per chunk, and the Zin chunk is staged in LDS as bf16
// hi/lo in the matching B-fragment order, double buffered, one workgroup
// barrier per chunk.  The A fragments of the next chunk are loaded while the
// current one is multiplied.  v_mfma_f32_32x32x16_bf16 lane layout: A lane l
// holds A[l % 32][8 (l / 32) + e], B lane l holds B[8 (l / 32) + e][l % 32],
// result register v of lane l is C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int kX3Chunk = 256;                         // K per chunk
constexpr int kX3StageBytes = 2 * 2 * (kX3Chunk / 8) * 32 * 16;  // [buffer][plane][k/8][column][8 bf16]

// round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <int KB, int NT>
__device__ __noinline__ void dense_x3(int64_t n, int64_t ld, const gbl<uint16_t>* __restrict__ Mhi,
                                      const gbl<uint16_t>* __restrict__ Mlo, const gbl<float>* __restrict__ Zin,
                                      int64_t row0, lds<float>* out, lds<char>* xs) {
  static_assert(NT == 512 && KB <= 32, "8 waves, at most 32 columns");
  constexpr int KC = kX3Chunk;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rt = wave & 1, kq = wave >> 1;
  const int li = lane & 31, h = lane >> 5;
  const int64_t arow = row0 + 32 * rt + li;
  const bool rowok = arow < n;
  const int nchunk = (int)((n + KC - 1) / KC);
  const gbl<uint16_t>* ph = Mhi + (rowok ? arow * ld : 0);
  const gbl<uint16_t>* pl = Mlo + (rowok ? arow * ld : 0);
  // A fragments of chunk c.  A chunk of a block whose rows and columns all lie
  // inside the matrix (the common case, uniform over the workgroup) is read
  // as four 16-byte loads at constant offsets from one address per plane.
  // Otherwise every 16-byte load reads inside the row (ld is a multiple of 8
  // and the group start is clamped below n), and elements past n or rows past
  // n are masked to zero afterwards.
  const bool block_in = row0 + 64 <= n;
  auto load_a = [&](int c, u16x8_t (&ah)[4], u16x8_t (&al)[4]) {
    const int64_t k0 = (int64_t)c * KC + kq * 64 + h * 32;
    if (block_in && (int64_t)(c + 1) * KC <= n) {
      const gbl<u16x8_t>* qh = reinterpret_cast<const gbl<u16x8_t>*>(ph + k0);
      const gbl<u16x8_t>* ql = reinterpret_cast<const gbl<u16x8_t>*>(pl + k0);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ah[s] = qh[s];
        al[s] = ql[s];
      }
      return;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t kk = k0 + 8 * s;
      const int64_t ka = kk < n ? kk : 0;
      ah[s] = *reinterpret_cast<const gbl<u16x8_t>*>(ph + ka);
      al[s] = *reinterpret_cast<const gbl<u16x8_t>*>(pl + ka);
      const int64_t left = rowok ? n - kk : 0;  // valid elements in this group
      if (left < 8) {  // rare: the K tail, or a row past n
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ah[s][e] = e < left ? ah[s][e] : (unsigned short)0;
          al[s][e] = e < left ? al[s][e] : (unsigned short)0;
        }
      }
    }
  };
  // staging of a Zin chunk: thread t < 32 * KB / 4 owns the 4 columns
  // 4 (t % (KB/4)) .. + 3 of the 8 rows of k-group t / (KB/4): 8 16-byte loads,
  // 4 columns x (hi, lo) fragments of 8 values written back
  constexpr int CG = KB / 4;  // column groups of 4
  const int scg = tid % CG, sg = tid / CG;
  const bool stager = tid < (KC / 8) * CG;
  auto load_b = [&](int c, f32x4_t (&zv)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t kk = (int64_t)c * KC + sg * 8 + e;
      const bool ok = stager && kk < n;
      const f32x4_t v = *reinterpret_cast<const gbl<f32x4_t>*>(Zin + (ok ? kk * KB + 4 * scg : 0));
      zv[e] = ok ? v : f32x4_t{};
    }
  };
  auto store_b = [&](int buf, const f32x4_t (&zv)[8]) {
    if (!stager) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u16x8_t hv, lv;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = zv[e][q];
        const unsigned short hb = bf16_rne(x);
        hv[e] = hb;
        lv[e] = bf16_rne(x - bf16_val(hb));
      }
      const int j = 4 * scg + q;
      *reinterpret_cast<lds<u16x8_t>*>(xs + (((buf * 2 + 0) * (KC / 8) + sg) * 32 + j) * 16) = hv;
      *reinterpret_cast<lds<u16x8_t>*>(xs + (((buf * 2 + 1) * (KC / 8) + sg) * 32 + j) * 16) = lv;
    }
  };
  f32x16_t acc = {};
  auto multiply = [&](int buf, const u16x8_t (&ah)[4], const u16x8_t (&al)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int g8 = kq * 8 + h * 4 + s;
      const u16x8_t bh = *reinterpret_cast<const lds<u16x8_t>*>(xs + (((buf * 2 + 0) * (KC / 8) + g8) * 32 + li) * 16);
      const u16x8_t bl = *reinterpret_cast<const lds<u16x8_t>*>(xs + (((buf * 2 + 1) * (KC / 8) + g8) * 32 + li) * 16);
      const bf16x8_t a1 = __builtin_bit_cast(bf16x8_t, ah[s]), a2 = __builtin_bit_cast(bf16x8_t, al[s]);
      const bf16x8_t b1 = __builtin_bit_cast(bf16x8_t, bh), b2 = __builtin_bit_cast(bf16x8_t, bl);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b2, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b1, acc, 0, 0, 0);
    }
  };
  // columns beyond KB of the staged fragments stay zero
  if constexpr (KB < 32)
    for (int e = tid; e < 2 * 2 * (KC / 8) * (32 - KB); e += NT) {
      const int j = KB + e % (32 - KB), rest = e / (32 - KB);
      *reinterpret_cast<lds<u16x8_t>*>(xs + (rest * 32 + j) * 16) = u16x8_t{};
    }
  u16x8_t ah0[4], al0[4], ah1[4], al1[4];
  f32x4_t zv[8];
  load_b(0, zv);
  load_a(0, ah0, al0);
  store_b(0, zv);
  __syncthreads();
  // Stage c: issue the loads of Zin chunk c + 1 and then of A chunk c + 1
  // (memory counters retire in order, so staging Zin waits for the Zin loads
  // only and the A loads stay in flight across the barrier), multiply chunk
  // c, stage Zin chunk c + 1 into LDS.  The prefetches past the last chunk
  // read valid, masked addresses and are discarded; they keep the loop free
  // of branches around the loads.
  int c = 0;
  auto stage = [&](const u16x8_t (&ah)[4], const u16x8_t (&al)[4], u16x8_t (&nh)[4], u16x8_t (&nl)[4]) {
    load_b(c + 1, zv);
    load_a(c + 1, nh, nl);
    multiply(c & 1, ah, al);
    store_b((c + 1) & 1, zv);
    __syncthreads();
    ++c;
  };
  while (true) {  // chunks in pairs so both register buffers are addressed statically
    stage(ah0, al0, ah1, al1);
    if (c >= nchunk) break;
    stage(ah1, al1, ah0, al0);
    if (c >= nchunk) break;
  }
  // sum the four K quarters of each row tile (the staging area is free now)
  lds<float>* red = reinterpret_cast<lds<float>*>(xs);  // 8 waves x 64 lanes x 16
#pragma unroll
  for (int v = 0; v < 16; ++v) red[(wave * 64 + lane) * 16 + v] = acc[v];
  __syncthreads();
  for (int e = tid; e < 64 * KB; e += NT) {
    const int rr = e / KB, j = e % KB;
    const int t = rr / 32, i = rr % 32;
    const int l = j + 32 * ((i / 4) % 2), v = 4 * (i / 8) + i % 4;
    float sum = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) sum += red[((t + 2 * q) * 64 + l) * 16 + v];
    out[e] = sum;
  }
}

// ---------------------------------------------------------------------------
// Factored minibatch gradient (quadratic measurements with the stochastic
// gradient estimate of Section 6):
//   G = (1/L) sum_{i in batch} w_i a_i a_i^T,   w_i = a_i^T X_t a_i - b_i,
// so Op Zin = A_B^T diag(w / L) (A_B Zin) takes two passes over the L x n
// minibatch A_B with a grid barrier between them:
//   factor_rows  one workgroup per minibatch row i: y_i = (w_i / L) a_i^T Zin
//   factor_cols  (in the apply's row blocks): (Op Zin)_j = sum_i a_ij y_i
// In sweep 1, Zin = B, so a_i^T V = (a_i^T B) Wb[:, :r] comes out of the same
// product and w_i = alpha ||a_i||^2 + sum_l d_l (a_i^T v_l)^2 - b_i is formed
// there.  The shift needs an upper bound on lambda_max(G):
//   G <= (1/L) sum_{w_i > 0} w_i a_i a_i^T = (1/L) A_+^T D A_+,
// whose nonzero eigenvalues are those of D^1/2 A_+ A_+^T D^1/2; Gershgorin's
// theorem on that L x L matrix gives
//   lambda_max(G) <= max_i sqrt(w_i+) sum_j |K_ij| sqrt(w_j+) / L,  K = A_B A_B^T,
// with |K_ij| widened by the rounding bound 2 n u ||a_i|| ||a_j||.  (The
// trace bound sum w_i+ ||a_i||^2 / L is tens of times larger for Gaussian
// measurements and would slow the subspace iteration accordingly.)
// ---------------------------------------------------------------------------
constexpr int kFacChunk = 256;  // minibatch rows staged per pass of factor_cols

template <typename T, int KB>
constexpr int fac_stage_bytes() {
  constexpr int cols = kFacChunk * KB * (int)sizeof(T) + kFacChunk * 8;  // y chunk + pool offsets
  constexpr int gram = 8 * 256 * (int)sizeof(T);                        // per-wave 16 x 16 tiles
  constexpr int shift = (2 * kMaxBatch + 16) * 8;                        // sqrt(w+), ||a|| sqrt(w+), maxima
  constexpr int rows = 9 * KB * (int)sizeof(T) + 128;
  constexpr int a = cols > gram ? cols : gram;
  constexpr int b = shift > rows ? shift : rows;
  return a > b ? a : b;
}

// pool row of a minibatch index, clamped into the pool (indices are checked
// when the context is created; the clamp keeps every access in bounds)
__device__ __forceinline__ int64_t pool_row(int v, int64_t m) {
  const int64_t q = v;
  return q < 0 ? 0 : (q >= m ? m - 1 : q);
}

typedef double f64x2_t __attribute__((ext_vector_type(2)));

// 16-byte load from global memory into 4 floats or 2 doubles
template <typename T>
__device__ __forceinline__ void vload_g(const gbl<T>* p, T* out) {
  if constexpr (sizeof(T) == 4) {
    const f32x4_t v = *reinterpret_cast<const gbl<f32x4_t>*>(p);
    out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
  } else {
    const f64x2_t v = *reinterpret_cast<const gbl<f64x2_t>*>(p);
    out[0] = v[0]; out[1] = v[1];
  }
}

// Phase 1 of a factored apply, minibatch rows i = wg, wg + nwg, ...
// t_i = a_i^T Zin (KB values) is accumulated by all threads over their
// elements of a_i, reduced within each wave by a transposing butterfly
// (each step halves the values a lane carries, so a wave needs KB - 1
// exchanges instead of 6 KB) and then over the waves in a fixed order.
template <typename T, int KB, int NT>
__device__ __noinline__ void factor_rows(int64_t n, int64_t lda, int64_t m, int L, const gbl<T>* __restrict__ A,
                                         const gbl<T>* __restrict__ bq, const gbl<int>* __restrict__ idx,
                                         const gbl<T>* __restrict__ Zin, gbl<T>* __restrict__ qy,
                                         gbl<double>* __restrict__ qw, gbl<double>* __restrict__ qn,
                                         const gbl<Ctl>* ctl, int r, bool first, lds<char>* scr, int wg, int nwg) {
  constexpr int VN = V16<T>::N;
  constexpr int WAVES = NT / 64;
  constexpr int GL = 64 / KB;  // lanes that share a column after the butterfly
  lds<T>* wsum = reinterpret_cast<lds<T>*>(scr);  // WAVES x KB
  lds<double>* sred = reinterpret_cast<lds<double>*>(scr + align16(WAVES * KB * (int)sizeof(T)));  // WAVES
  lds<T>* tv = reinterpret_cast<lds<T>*>(scr + align16(WAVES * KB * (int)sizeof(T)) + 8 * WAVES);   // KB
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = wg; i < L; i += nwg) {
    const int64_t prow = pool_row(idx[i], m);
    const gbl<T>* a = A + prow * lda;
    T acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0;
    double sa = 0.0;
    // GU groups of VN elements per iteration, all their loads issued first
    // (GU = 2 spills at k = 16; the compiler overlaps iterations by itself)
    constexpr int GU = 1;
    for (int64_t j0 = (int64_t)VN * tid; j0 < n; j0 += (int64_t)GU * VN * NT) {
      T av[GU][VN];
      T z[GU][VN][KB];
#pragma unroll
      for (int h = 0; h < GU; ++h) {
        const int64_t jh = j0 + (int64_t)h * VN * NT;
        if (jh + VN <= n) {
          vload_g<T>(a + jh, av[h]);
        } else {
#pragma unroll
          for (int e = 0; e < VN; ++e) av[h][e] = (jh + e < n) ? a[jh + e] : (T)0;
        }
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          const int64_t j = (jh + e < n) ? jh + e : n - 1;  // av = 0 past n
#pragma unroll
          for (int q = 0; q < KB / VN; ++q) vload_g<T>(Zin + j * KB + q * VN, z[h][e] + q * VN);
        }
      }
#pragma unroll
      for (int h = 0; h < GU; ++h)
#pragma unroll
        for (int e = 0; e < VN; ++e) {
#pragma unroll
          for (int c = 0; c < KB; ++c) acc[c] += av[h][e] * z[h][e][c];
          sa += (double)av[h][e] * (double)av[h][e];
        }
    }
#pragma unroll
    for (int st = 0; (KB >> st) > 1; ++st) {
      const int h = KB >> (st + 1), o = 32 >> st;
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const T keep = up ? acc[q + h] : acc[q];
        const T send = up ? acc[q] : acc[q + h];
        acc[q] = keep + __shfl_xor(send, o, 64);
      }
    }
    const T colsum = group_sum<GL>(acc[0]);  // column lane / GL of this wave's partial
    if (lane % GL == 0) wsum[wave * KB + lane / GL] = colsum;
    sa = wave_sum(sa);
    if (lane == 0) sred[wave] = sa;
    __syncthreads();
    if (tid < KB) {
      T s = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) s += wsum[w * KB + tid];
      tv[tid] = s;
    }
    __syncthreads();
    if (tid < 64) {
      double w;
      if (first) {
        double na = 0.0;
#pragma unroll
        for (int q = 0; q < WAVES; ++q) na += sred[q];
        double vl = 0.0;  // (a_i^T V)_l = sum_c t_c Wb[c][l]
        if (lane < r)
#pragma unroll 4
          for (int c = 0; c < KB; ++c) vl += (double)tv[c] * ctl->Wb[c * KB + lane];
        const double dl = (lane < r) ? ctl->d[lane] : 0.0;
        const double x = ctl->alpha * na + wave_sum(dl * vl * vl);
        w = x - (double)bq[prow];
        if (lane == 0) {
          qw[i] = w;
          qn[i] = na;
        }
      } else {
        w = qw[i];
      }
      if (lane < KB) qy[(int64_t)i * KB + lane] = (T)((w / (double)L) * (double)tv[lane]);
    }
    __syncthreads();  // the scratch is reused by the next row
  }
}

// v_mfma_{f32,f64}_16x16x4: A lane l holds A[l % 16][l / 16], B lane l holds
// B[l / 16][l % 16]; result register v of lane l is row mfma16_row(l / 16, v),
// column l % 16.
template <typename T>
__device__ __forceinline__ int mfma16_row(int kq, int v) {
  if constexpr (sizeof(T) == 8) return kq + 4 * v;
  else return 4 * kq + v;
}

// Minibatch Gram matrix K = A_B A_B^T (sweep 1): 16 x 16 tiles (I, J), I <= J,
// spread over the workgroups; each wave takes every WAVES-th K chunk of the
// contraction, the waves' tiles are summed in a fixed order, and both K_IJ
// and K_JI are stored.  A lane reads 16 contiguous bytes of its row per
// chunk; within a chunk the K = 4 products take its elements in turn, the
// same permutation of columns for both operands.
template <typename T, int NT>
__device__ __noinline__ void factor_gram(int64_t n, int64_t lda, int64_t m, int L, const gbl<T>* __restrict__ A,
                                         const gbl<int>* __restrict__ idx, gbl<T>* __restrict__ qk, lds<T>* red,
                                         int wg, int nwg) {
  constexpr int VN = V16<T>::N;
  constexpr int CW = 4 * VN;  // columns per chunk
  constexpr int WAVES = NT / 64;
  using AccT = typename std::conditional<sizeof(T) == 8, f64x4_t, f32x4_t>::type;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int nt = (L + 15) / 16;
  const int ntiles = nt * (nt + 1) / 2;
  const int64_t nch = (n + CW - 1) / CW;
  for (int tau = wg; tau < ntiles; tau += nwg) {
    int I = 0, rem = tau;
    while (rem >= nt - I) {
      rem -= nt - I;
      ++I;
    }
    const int J = I + rem;
    const int ri = 16 * I + li, rj = 16 * J + li;
    const T mi = ri < L ? (T)1 : (T)0, mj = rj < L ? (T)1 : (T)0;
    const gbl<T>* pa = A + pool_row(idx[ri < L ? ri : 0], m) * lda;
    const gbl<T>* pb = A + pool_row(idx[rj < L ? rj : 0], m) * lda;
    AccT acc = {};
    for (int64_t ch = wave; ch < nch; ch += WAVES) {
      const int64_t k0 = ch * CW + VN * kq;
      T va[VN], vb[VN];
      if (ch * CW + CW <= n) {
        vload_g<T>(pa + k0, va);
        vload_g<T>(pb + k0, vb);
      } else {
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          va[e] = (k0 + e < n) ? pa[k0 + e] : (T)0;
          vb[e] = (k0 + e < n) ? pb[k0 + e] : (T)0;
        }
      }
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        if constexpr (sizeof(T) == 8)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[e] * mi, vb[e] * mj, acc, 0, 0, 0);
        else
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(va[e] * mi, vb[e] * mj, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave * 256 + mfma16_row<T>(kq, v) * 16 + li] = acc[v];
    __syncthreads();
    for (int e = tid; e < 256; e += NT) {
      T s = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) s += red[w * 256 + e];
      const int gi = 16 * I + e / 16, gj = 16 * J + e % 16;
      if (gi < L && gj < L) {
        qk[(int64_t)gi * L + gj] = s;
        if (I != J) qk[(int64_t)gj * L + gi] = s;
      }
    }
    __syncthreads();
  }
}

// Upper bound on lambda_max(G) for the shift (see above), from K, w and
// ||a_i||^2; all threads of one workgroup, every thread gets the result.
template <typename T, int NT>
__device__ __noinline__ double factor_shift(int64_t n, int L, double unit_round, const gbl<T>* __restrict__ qk,
                                            const gbl<double>* __restrict__ qw, const gbl<double>* __restrict__ qn,
                                            lds<double>* s) {
  constexpr int WAVES = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  lds<double>* sw = s;         // sqrt(w_i+)
  lds<double>* sv = s + L;     // ||a_i|| sqrt(w_i+)
  lds<double>* misc = s + 2 * L;
  for (int i = tid; i < L; i += NT) {
    const double wp = sqrt(fmax(qw[i], 0.0));
    sw[i] = wp;
    sv[i] = sqrt(qn[i]) * wp;
  }
  __syncthreads();
  if (wave == 0) {
    double a = 0.0;
    for (int i = lane; i < L; i += 64) a += sv[i];
    a = wave_sum(a);
    if (lane == 0) misc[0] = a;
  }
  __syncthreads();
  const double S = misc[0];
  const double gam = 2.0 * (double)n * unit_round;  // |fl(K_ij) - K_ij| <= gam ||a_i|| ||a_j||
  double mx = 0.0;
  for (int i = tid; i < L; i += NT) {
    if (sw[i] > 0.0) {
      const gbl<T>* row = qk + (int64_t)i * L;
      double acc = 0.0;
#pragma unroll 16
      for (int j = 0; j < L; ++j) acc += fabs((double)row[j]) * sw[j];
      mx = fmax(mx, sw[i] * (acc + gam * sqrt(qn[i]) * S));
    }
  }
  mx = wave_max(mx);
  if (lane == 0) misc[1 + wave] = mx;
  __syncthreads();
  double g = 0.0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) g = fmax(g, misc[1 + w]);
  return g / (double)L;
}

// Phase 2 of a factored apply for the rows row0 .. row0 + ROWS - 1:
// out[j][c] = sum_i a_i[row0 + j] y_i[c].  Thread (slice sl, row j) takes
// the minibatch rows i = sl (mod NT / ROWS); a wave's load covers two
// contiguous ROWS-element pieces of two pool rows.  The y_i are staged in LDS
// in chunks; the slices are summed in a fixed order.
template <typename T, int KB, int ROWS, int NT>
__device__ __noinline__ void factor_cols(int64_t n, int64_t lda, int64_t m, int L, const gbl<T>* __restrict__ A,
                                         const gbl<int>* __restrict__ idx, const gbl<T>* __restrict__ qy,
                                         int64_t row0, lds<T>* out, lds<char>* scr) {
  static_assert(ROWS == 32, "two slices per wave");
  constexpr int SL = NT / ROWS;
  constexpr int CH = kFacChunk;
  constexpr int WAVES = NT / 64;
  lds<T>* ys = reinterpret_cast<lds<T>*>(scr);                                     // CH x KB
  lds<int64_t>* is = reinterpret_cast<lds<int64_t>*>(scr + CH * KB * (int)sizeof(T));  // CH pool offsets
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = tid % ROWS, sl = tid / ROWS;
  const bool rowok = row0 + j < n;
  const int64_t col = rowok ? row0 + j : 0;
  const T msk = rowok ? (T)1 : (T)0;
  T acc[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) acc[c] = 0;
  for (int i0 = 0; i0 < L; i0 += CH) {
    const int cnt = (L - i0 < CH) ? L - i0 : CH;
    __syncthreads();
    for (int e = tid; e < cnt * KB; e += NT) ys[e] = qy[(int64_t)i0 * KB + e];
    for (int e = tid; e < cnt; e += NT) is[e] = pool_row(idx[i0 + e], m) * lda;
    __syncthreads();
    // UB loads in flight per thread (all of a 256-row chunk's share at
    // NT / ROWS = 16 slices), clamped into the chunk and masked past its end
    constexpr int UB = CH / SL;
    for (int ii = sl; ii < cnt; ii += UB * SL) {
      T a[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int iu = ii + u * SL;
        const bool ok = iu < cnt;
        a[u] = A[is[ok ? iu : cnt - 1] + col] * (ok ? msk : (T)0);
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int iu = ii + u * SL < cnt ? ii + u * SL : cnt - 1;
#pragma unroll
        for (int c = 0; c < KB; ++c) acc[c] += a[u] * ys[iu * KB + c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < KB; ++c) acc[c] += __shfl_xor(acc[c], 32, 64);  // slices 2w and 2w + 1
  __syncthreads();
  lds<T>* red = reinterpret_cast<lds<T>*>(scr);  // WAVES x ROWS x KB
  if (lane < 32)
#pragma unroll
    for (int c = 0; c < KB; ++c) red[(wave * ROWS + j) * KB + c] = acc[c];
  __syncthreads();
  for (int e = tid; e < ROWS * KB; e += NT) {
    T s = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) s += red[w * ROWS * KB + e];
    out[e] = s;
  }
}

// ---------------------------------------------------------------------------
// apply phase: Zout = Yhat Q for the sweep basis Q = Zin W, over all row
// blocks of this workgroup:
//   Zout_i = (opscale (Op Zin)_i + sdiag Zin_i) W + V_i diag(ceff) PW,
//   V_i = (B_i Wb)[:, :r],  PW = V^T Q,
// with the FP64 Gram partials Zin^T Zout, Zout^T Zout, V^T Zout -> part[wg].
// GRAD (masked objective, first sweep, where Zin = B): the gradient value
// g_e = X_ij - M_ij is formed from the same gathered row j, as
//   X_ij = alpha [i == j] + V_i diag(d) V_j^T = alpha [i == j] + B_j w_i,
//   w_i = Wb[:, :r] diag(d) V_i^T,
// stored for the later sweeps and used at once; sum g_e^2 and sum X_ij^2
// over Omega go to part[wg * PSTRIDE + PLEN], part[wg * PSTRIDE + PLEN + 1].
// ---------------------------------------------------------------------------
template <typename T, int KB, int OPK, int NT, bool GRAD, bool CACHE>
__device__ void apply_phase(const Cfg& cfg, const Ctl* ctl, const Data<T>& dat, const T* __restrict__ gv,
                            T* __restrict__ gout, const T* __restrict__ B, const T* __restrict__ Zin,
                            T* __restrict__ Zout, const T* Zprev, double* part, double* smem,
                            const CsrCache<T>& cc, lds<char>* xs, Team tm) {
  using SH = StepShape<T, KB, OPK, NT>;
  constexpr int ROWS = SH::ROWS, RPW = SH::RPW;
  using SM = ApplySmem<T, KB, ROWS, SH::GWROWS>;
  constexpr int LD = SM::LD;
  constexpr int VN = V16<T>::N;
  constexpr int WAVES = NT / 64;
  constexpr int SE = (ROWS * KB + NT - 1) / NT;  // staged elements per thread
  static_assert(!GRAD || OPK == OP_CSR, "the fused gradient is the masked (CSR) objective's");
  T* tb = reinterpret_cast<T*>(smem + SM::ACC);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = cfg.r;
  const int64_t n = cfg.n;
  // explicit residuals of the previous Rayleigh-Ritz sweep: this sweep's
  // input Zin is that sweep's output, Zprev its input
  const bool xr = SM::XR && cfg.xres && ctl->xvalid;
  // per-sweep coefficients: loaded into registers here, stored to LDS with
  // the first row block's loads in flight (before that block's barrier, the
  // first point of use), so the two round trips to memory overlap
  constexpr int CPT = (KB * KB + NT - 1) / NT;  // coefficient entries per thread
  T cw[CPT], cwb[CPT], cpw[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    const int e = tid + u * NT;
    cw[u] = 0;
    cwb[u] = 0;
    cpw[u] = 0;
    if (e < KB * KB) {
      cw[u] = (T)ctl->W[e];
      cwb[u] = (T)ctl->Wb[e];
      cpw[u] = (e / KB < r) ? (T)ctl->PW[e] : (T)0;
    }
  }
  // Chebyshev filter of the sweep (degree 1 on the interval [0, b] of the
  // unwanted spectrum, b = cheb_b; 0: none): Zout = fa Yhat Q + fb Q with
  // fa = 2/b, fb = -1, folded into the operator's coefficients
  const double chb = ctl->cheb_b;
  const double fa = chb > 0.0 ? 2.0 / chb : 1.0, fb = chb > 0.0 ? -1.0 : 0.0;
  const double ce = tid < KB ? ctl->ceff[tid] : 0.0;
  auto store_coefs = [&]() {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int e = tid + u * NT, i = e / KB, j = e % KB;
      if (e < KB * KB) {
        tb[SM::T_W + i * LD + j] = cw[u];
        tb[SM::T_WB + i * LD + j] = cwb[u];
        tb[SM::T_PW + e] = cpw[u];
      }
    }
    if (tid < KB) tb[SM::T_CE + tid] = (T)(fa * ce);
  };
  for (int e = tid; e < SM::ACC; e += NT) smem[e] = 0.0;
  const T opscale = (T)(fa * ctl->opscale), sdiag = (T)(fa * ctl->sdiag + fb);
  T alpha = 0, dl = 0;
  if constexpr (GRAD) {
    alpha = (T)ctl->alpha;
    dl = (lane < r) ? (T)ctl->d[lane] : (T)0;
  }
  double accg = 0.0, accx = 0.0;  // GRAD: sums of g^2 and X_ij^2 over this lane's nonzeros
  const int64_t nblk = (n + ROWS - 1) / ROWS;
  int jb = 0;  // this workgroup's block counter (cache position)
  for (int64_t blk = tm.wg; blk < nblk; blk += tm.nwg, ++jb) {
    const int64_t row0 = blk * ROWS;
    // this block's rows of Zin and B: loads issued now, stored to LDS after
    // the gathers below (their latency overlaps)
    T pz[SE], pb[SE], pp[SE];
#pragma unroll
    for (int u = 0; u < SE; ++u) {
      const int e = tid + u * NT;
      const int64_t i = row0 + e / KB;
      pz[u] = 0;
      pb[u] = 0;
      pp[u] = 0;
      if (e < ROWS * KB && i < n) {
        pz[u] = Zin[i * KB + e % KB];
        pb[u] = B[i * KB + e % KB];
        // Zprev may be the block this sweep writes (its row i is read here,
        // before this block's rows are written, and by no other workgroup)
        if (SM::XR && xr) pp[u] = Zprev[i * KB + e % KB];
      }
    }
    if (jb == 0) store_coefs();
    __syncthreads();  // previous block's LDS reads are done; coefficients are visible
    if constexpr (OPK == OP_CSR) {
      // RPW rows per wave, gathered together; a row's nonzeros are split over
      // lane groups of LPN lanes, each lane owning a 16-byte chunk of the
      // gathered row.  U slots of NPI nonzeros per row are in flight per
      // iteration, and the next iteration's column indices and values are
      // fetched before this one's rows are used.
      constexpr int LPN = KB / VN;
      constexpr int NPI = 64 / LPN;
      constexpr int U = 8 / RPW;
      constexpr int STEP = NPI * U;
      const int sub = lane % LPN, grp = lane / LPN;
      const T* wsrc = GRAD ? dat.val : gv;  // M_Omega (GRAD) or the stored gradient
      // entry e's column index and value: cache positions (CACHE) or global
      auto ld_col = [&](int e) -> int {
        if constexpr (CACHE) return cc.col[e]; else return dat.col[e];
      };
      auto ld_w = [&](int e) -> T {
        if constexpr (CACHE) return GRAD ? cc.val[e] : cc.gv[e]; else return wsrc[e];
      };
      int64_t iq[RPW];
      int e0[RPW], e1[RPW];
      int nit = 0;
#pragma unroll
      for (int q = 0; q < RPW; ++q) {
        iq[q] = row0 + wave * RPW + q;
        e0[q] = 0;
        e1[q] = 0;
        if (iq[q] < n) {  // uniform per wave
          if constexpr (CACHE) {
            e0[q] = cc.rloc[jb * (ROWS + 1) + wave * RPW + q];
            e1[q] = cc.rloc[jb * (ROWS + 1) + wave * RPW + q + 1];
          } else {
            e0[q] = dat.rp[iq[q]];
            e1[q] = dat.rp[iq[q] + 1];
          }
        }
        nit = max(nit, (e1[q] - e0[q] + STEP - 1) / STEP);
      }
      T bi[RPW];
      if constexpr (GRAD) {
#pragma unroll
        for (int q = 0; q < RPW; ++q) bi[q] = (lane < KB && iq[q] < n) ? B[iq[q] * KB + lane] : (T)0;
      }
      int jn[RPW][U];
      T wn[RPW][U];
#pragma unroll
      for (int q = 0; q < RPW; ++q)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int eu = e0[q] + grp + u * NPI;
          const bool ok = eu < e1[q];
          jn[q][u] = ok ? ld_col(eu) : 0;  // in-range row, weight 0
          wn[q][u] = ok ? ld_w(eu) : (T)0;
        }
      T wd[RPW][VN];  // GRAD: this lane's chunk of w_i
      if constexpr (GRAD) {
        // w_i = Wb[:, :r] diag(d) (B_i Wb[:, :r])^T in this wave's scratch
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
          T* gw = tb + SM::T_GW + (wave * RPW + q) * 3 * KB;
          if (lane < KB) gw[lane] = bi[q];
        }
        wsync();
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
          T* gw = tb + SM::T_GW + (wave * RPW + q) * 3 * KB;
          if (lane < KB) {
            T v = 0;
            if (lane < r)
#pragma unroll 8
              for (int c = 0; c < KB; ++c) v += gw[c] * tb[SM::T_WB + c * LD + lane];
            gw[KB + lane] = v * dl;  // V_il d_l, zero for l >= r
          }
        }
        wsync();
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
          T* gw = tb + SM::T_GW + (wave * RPW + q) * 3 * KB;
          if (lane < KB) {
            T w = 0;
            for (int l = 0; l < r; ++l) w += tb[SM::T_WB + lane * LD + l] * gw[KB + l];
            gw[2 * KB + lane] = w;
          }
        }
        wsync();
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
          const T* gw = tb + SM::T_GW + (wave * RPW + q) * 3 * KB;
#pragma unroll
          for (int v = 0; v < VN; ++v) wd[q][v] = gw[2 * KB + sub * VN + v];
        }
      }
      T acc[RPW][VN];
#pragma unroll
      for (int q = 0; q < RPW; ++q)
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[q][v] = 0;
      for (int it = 0; it < nit; ++it) {  // same trip count for all lanes of the wave
        int jj[RPW][U];
        T ww[RPW][U];
#pragma unroll
        for (int q = 0; q < RPW; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            jj[q][u] = jn[q][u];
            ww[q][u] = wn[q][u];
          }
        T z[RPW][U][VN];
#pragma unroll
        for (int q = 0; q < RPW; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) vload<T>(Zin + (int64_t)jj[q][u] * KB + sub * VN, z[q][u]);
#pragma unroll
        for (int q = 0; q < RPW; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int eu = e0[q] + (it + 1) * STEP + grp + u * NPI;
            const bool ok = eu < e1[q];
            jn[q][u] = ok ? ld_col(eu) : 0;
            wn[q][u] = ok ? ld_w(eu) : (T)0;
          }
#pragma unroll
        for (int q = 0; q < RPW; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            T w = ww[q][u];
            if constexpr (GRAD) {
              T x = 0;
#pragma unroll
              for (int v = 0; v < VN; ++v) x += wd[q][v] * z[q][u][v];
              x = group_sum<LPN>(x);
              if (jj[q][u] == iq[q]) x += alpha;
              const int eu = e0[q] + it * STEP + grp + u * NPI;
              const bool ok = eu < e1[q];
              const T gval = x - w;
              w = ok ? gval : (T)0;
              if (ok && sub == 0) {
                if constexpr (CACHE) cc.g[eu] = gval; else gout[eu] = gval;
                accg += (double)gval * (double)gval;
                accx += (double)x * (double)x;
              }
            }
#pragma unroll
            for (int v = 0; v < VN; ++v) acc[q][v] += w * z[q][u][v];
          }
      }
#pragma unroll
      for (int q = 0; q < RPW; ++q) {
#pragma unroll
        for (int o = LPN; o < 64; o <<= 1)
#pragma unroll
          for (int v = 0; v < VN; ++v) acc[q][v] += __shfl_xor(acc[q][v], o, 64);
        if (grp == 0) {
#pragma unroll
          for (int v = 0; v < VN; ++v) tb[SM::T_U + (wave * RPW + q) * KB + sub * VN + v] = acc[q][v];
        }
      }
    } else if constexpr (OPK == OP_FACTOR) {
      factor_cols<T, KB, ROWS, NT>(n, cfg.lda, cfg.m, cfg.batch, (const gbl<T>*)dat.A, (const gbl<int>*)dat.bidx,
                                   (const gbl<T>*)dat.qy, row0, (lds<T>*)(tb + SM::T_U), xs);
    } else if constexpr (OPK == OP_DENSE_X3) {
      static_assert(ROWS == 64, "two 32-row tiles per block");
      static_assert(sizeof(T) == 4, "float state");
      dense_x3<KB, NT>(n, cfg.ld, (const gbl<uint16_t>*)dat.Dhi, (const gbl<uint16_t>*)dat.Dlo,
                       (const gbl<float>*)Zin, row0, (lds<float>*)(tb + SM::T_U), xs);
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
#pragma unroll
    for (int u = 0; u < SE; ++u) {
      const int e = tid + u * NT;
      if (e < ROWS * KB) {
        tb[SM::T_ZIN + e] = pz[u];
        tb[SM::T_B + e] = pb[u];
      }
    }
    __syncthreads();
    // V_i = (B_i Wb)[:, :r] and y_i = opscale (Op Zin)_i + sdiag Zin_i
    for (int e = tid; e < ROWS * KB; e += NT) {
      const int rr = e / KB, l = e % KB;
      T v = 0;
      if (l < r)
#pragma unroll 8
        for (int q = 0; q < KB; ++q) v += tb[SM::T_B + rr * KB + q] * tb[SM::T_WB + q * LD + l];
      tb[SM::T_V + e] = v;
      tb[SM::T_ZO + e] = opscale * tb[SM::T_U + e] + sdiag * tb[SM::T_ZIN + e];
    }
    __syncthreads();
    // z_i = y_i W + V_i diag(ceff) PW (rows beyond n are zero)
    for (int e = tid; e < ROWS * KB; e += NT) {
      const int rr = e / KB, c = e % KB;
      T z = 0;
#pragma unroll 8
      for (int a = 0; a < KB; ++a) z += tb[SM::T_ZO + rr * KB + a] * tb[SM::T_W + a * LD + c];
      for (int l = 0; l < r; ++l) z += tb[SM::T_V + rr * KB + l] * tb[SM::T_CE + l] * tb[SM::T_PW + l * KB + c];
      const int64_t i = row0 + rr;
      if (i < n) Zout[i * KB + c] = z; else z = 0;
      tb[SM::T_U + e] = z;
    }
    __syncthreads();
    if (SM::XR && xr) {
      // residual block of the previous sweep's Ritz pairs, row-wise:
      // Zin_i S - Zprev_i (W S Theta) (zero beyond n); S and W S Theta are
      // read from the control block (L2), Zprev's rows take the T_B rows
#pragma unroll
      for (int u = 0; u < SE; ++u) {
        const int e = tid + u * NT;
        if (e < ROWS * KB) tb[SM::T_B + e] = pp[u];
      }
      __syncthreads();
      for (int e = tid; e < ROWS * KB; e += NT) {
        const int rr = e / KB, c = e % KB;
        T v = 0;
#pragma unroll 8
        for (int a = 0; a < KB; ++a)
          v += tb[SM::T_ZIN + rr * KB + a] * (T)ctl->XS[a * KB + c] - tb[SM::T_B + rr * KB + a] * (T)ctl->XWT[a * KB + c];
        tb[SM::T_ZO + e] = v;
      }
      __syncthreads();
    }
    // FP64 Gram partials (products of working-precision values are exact)
    for (int e = tid; e < KB * KB; e += NT) {
      const int a = e / KB, c = e % KB;
      double cz = 0.0, gg = 0.0, p = 0.0;
#pragma unroll 4
      for (int rr = 0; rr < ROWS; ++rr) {
        const double zb = (double)tb[SM::T_U + rr * KB + c];
        cz += (double)tb[SM::T_ZIN + rr * KB + a] * zb;
        gg += (double)tb[SM::T_U + rr * KB + a] * zb;
        p += (double)tb[SM::T_V + rr * KB + a] * zb;
      }
      smem[e] += cz;
      smem[KB * KB + e] += gg;
      smem[2 * KB * KB + e] += p;
      if (SM::XR && xr && e < KB) {
        double q = 0.0;
        for (int rr = 0; rr < ROWS; ++rr) {
          const double v = (double)tb[SM::T_ZO + rr * KB + e];
          q += v * v;
        }
        smem[SM::PLEN + e] += q;
      }
    }
  }
  // the objective's partials, in a fixed order (waves, then lanes)
  double* sred = reinterpret_cast<double*>(tb);  // the typed area is free now
  __syncthreads();
  if constexpr (GRAD) {
    accg = wave_sum(accg);
    accx = wave_sum(accx);
    if (lane == 0) {
      sred[wave] = accg;
      sred[WAVES + wave] = accx;
    }
  }
  __syncthreads();
  // the record (PartRec): C, G's upper triangle, P's r rows, the
  // objective's two sums, the residuals' column sums
  using PR = PartRec<KB>;
  double* dst = part + (size_t)tm.wg * PR::len(r, SM::XR != 0);
  for (int e = tid; e < KB * KB; e += NT) {
    dst[e] = smem[e];
    const int a = e / KB, c = e % KB;
    if (a <= c) dst[PR::G_OFF + PR::tri(a, c)] = smem[KB * KB + e];
  }
  for (int e = tid; e < r * KB; e += NT) dst[PR::P_OFF + e] = smem[2 * KB * KB + e];
  if (tid == 0) {
    double sg = 0.0, sx = 0.0;
    if constexpr (GRAD)
      for (int w = 0; w < WAVES; ++w) {
        sg += sred[w];
        sx += sred[WAVES + w];
      }
    dst[PR::f_off(r)] = sg;
    dst[PR::f_off(r) + 1] = sx;
  }
  if constexpr (SM::XR != 0)
    if (tid < KB) dst[PR::x_off(r) + tid] = xr ? smem[SM::PLEN + tid] : 0.0;
}

// ---------------------------------------------------------------------------
// Gram partial B^T B of a basis block -> part[wg] (KB x KB), for the
// orthonormalising transform of a freshly uploaded basis.
// ---------------------------------------------------------------------------
template <typename T, int KB, int GROWS, int NT>
__device__ __noinline__ void gram_phase(const Cfg& cfg, const gbl<T>* Bm, gbl<double>* part, lds<double>* smem) {
  lds<double>* acc = smem;                                   // KB * KB
  lds<T>* rows = reinterpret_cast<lds<T>*>(smem + KB * KB);  // GROWS x KB
  const int tid = threadIdx.x;
  const int64_t n = cfg.n;
  for (int e = tid; e < KB * KB; e += NT) acc[e] = 0.0;
  const int64_t nblk = (n + GROWS - 1) / GROWS;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t row0 = blk * GROWS;
    __syncthreads();
    for (int e = tid; e < GROWS * KB; e += NT) {
      const int64_t i = row0 + e / KB;
      rows[e] = (i < n) ? Bm[i * KB + e % KB] : (T)0;
    }
    __syncthreads();
    for (int e = tid; e < KB * KB; e += NT) {
      const int a = e / KB, c = e % KB;
      double s = 0.0;
#pragma unroll 4
      for (int rr = 0; rr < GROWS; ++rr) s += (double)rows[rr * KB + a] * (double)rows[rr * KB + c];
      acc[e] += s;
    }
  }
  __syncthreads();
  gbl<double>* dst = part + (size_t)blockIdx.x * KB * KB;
  for (int e = tid; e < KB * KB; e += NT) dst[e] = acc[e];
}

template <typename T>
__device__ __forceinline__ T* zbuf(T* Z0, T* Z1, T* Z2, int i) {
  return i == 0 ? Z0 : (i == 1 ? Z1 : Z2);
}

__device__ __forceinline__ int ldi(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ldi64(const int64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Orders this workgroup's earlier global writes before its later reads
// (values one lane of the serial wavefront wrote and another reads).
__device__ __forceinline__ void wg_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void stamp(const Bufs& b, int slot) {
  if (b.ts && threadIdx.x == 0) b.ts[slot] = wall_clock64();
}

// per-workgroup stamp of sweep s (1-based), e = 0 start, 1 arrival at its barrier
__device__ __forceinline__ void stamp_wg(const Bufs& b, Team tm, int s, int e) {
  if (b.ts && threadIdx.x == 0 && s <= kTsWgSweeps)
    b.ts[kTsWg + (2 * (s - 1) + e) * tm.nwg + tm.wg] = wall_clock64();
}

// ---------------------------------------------------------------------------
// persistent step kernel: `nsteps` iterations of Algorithm 2.  Launched
// cooperatively (all workgroups resident).  One grid barrier per sweep; its
// Gram partials are summed on the way through the barrier, and the small
// solve of the step's last sweep also ends the step (next basis, iterate,
// certificate, step scalars).
// ---------------------------------------------------------------------------
// Static LDS of the step: the apply's typed scratch and partials (smem), and
// the staging area of the matrix-core and factored applies (xstage).
template <typename T, int KB, int OPK, int NT>
struct StepLds {
  using SH = StepShape<T, KB, OPK, NT>;
  using SM = ApplySmem<T, KB, SH::ROWS, SH::GWROWS>;
  static constexpr int DENSE_STAGE = (OPK == OP_DENSE) ? (64 * (KB + 1) * (int)sizeof(T) + 7) / 8 : 0;
  static constexpr int SMEM_DOUBLES = SM::TOTAL + DENSE_STAGE;
  static constexpr int XSTAGE_BYTES =
      OPK == OP_DENSE_X3 ? kX3StageBytes : (OPK == OP_FACTOR ? fac_stage_bytes<T, KB>() : 16);
};

// `nsteps` iterations of one instance by the team `tm` (the body of k_step
// and of each team of k_serve).  With a deadline (device wall clock, 0:
// none) the team also stops at the first step boundary past it: the
// workgroup that ends a step compares the clock and marks the instance
// paused for launch `seq`, which every workgroup of the team reads after the
// barrier, so the team decides as one.
template <typename T, int KB, int OPK, int NT, bool CACHE>
__device__ __forceinline__ void step_loop(const Cfg& cfg, Ctl* __restrict__ ctl, const Data<T>& dat,
                                          T* __restrict__ Z0, T* __restrict__ Z1, T* __restrict__ Z2,
                                          T* __restrict__ g, const Bufs& b, int nsteps, Team tm, double* smem,
                                          char* xstage, char* dyn, long long deadline = 0, int64_t seq = 0) {
  using SH = StepShape<T, KB, OPK, NT>;
  using SM = ApplySmem<T, KB, SH::ROWS, SH::GWROWS>;
  static_assert(!CACHE || OPK == OP_CSR, "the LDS cache holds CSR data");
  const int tid = threadIdx.x;

  const bool masked = cfg.kind == MASKED_CSR;
  lds<double>* lsums = (lds<double>*)(smem + SM::SUMS);  // the barrier's reduced record
  // the configuration in LDS for the small solve, a function of its own that
  // would otherwise read each field from argument memory, one round trip at
  // a time
  __shared__ Cfg s_cfg;
  if (tid == 0) s_cfg = cfg;
  __syncthreads();
  CsrCache<T> cc{};
  if constexpr (CACHE) {
    const CacheLayout L = cache_layout(cfg.cache_blocks, SH::ROWS, cfg.cache_nnz, (int)sizeof(T), masked);
    cc.rloc = (lds<int>*)(dyn + L.rloc);
    cc.col = (lds<int>*)(dyn + L.col);
    cc.val = (lds<T>*)(dyn + L.val);
    cc.g = (lds<T>*)(dyn + L.g);
    cc.gv = masked ? cc.g : cc.val;
    load_csr_cache<T, SH::ROWS, NT>(cfg, dat, cc, tm);
  }
  // The launch's first step reads the control words (read together, one
  // round trip); every later step takes them from the tag of the barrier
  // that ended the previous one (kSweep*: its input block, and whether the
  // team stops), so no step waits on a read of ctl before its first loads.
  int src = ldi(&ctl->src);
  {
    const int stop = ldi(&ctl->stop), status = ldi(&ctl->status);
    const int64_t pause = deadline != 0 ? ldi64(&ctl->pause_seq) : seq - 1;
    if ((stop | status) != 0 || pause == seq) return;
  }
  for (int st = 0; st < nsteps; ++st) {
    // the step scalars (shift, coefficients) and the basis (B, Wb) were set
    // at the end of the previous iteration
    int64_t t0 = 0;
    if constexpr (OPK == OP_FACTOR) t0 = ldi64(&ctl->t);
    if (tm.wg == 0) {
      stamp(b, 0);
      stamp(b, 1);  // no separate gradient phase: it is part of sweep 1
    }
    const int o1 = (src + 1) % 3, o2 = (src + 2) % 3;
    const T* Bm = zbuf(Z0, Z1, Z2, src);
    const T* gvals = masked ? g : dat.val;
    Data<T> dstep = dat;
    if constexpr (OPK == OP_FACTOR) {  // this step's minibatch: row (t - 1) mod batch_steps
      const int64_t bs = cfg.batch_steps;
      dstep.bidx = dat.bidx + (((t0 - 1) % bs + bs) % bs) * cfg.batch;
    }
    for (int s = 1; s <= cfg.max_inner; ++s) {
      const int in = (s == 1) ? src : ((s % 2 == 0) ? o1 : o2);
      const int out = (s % 2 == 1) ? o1 : o2;
      const bool grad = masked && s == 1;
      T* Zin = zbuf(Z0, Z1, Z2, in);
      T* Zout = zbuf(Z0, Z1, Z2, out);
      // the previous sweep's input (explicit residuals; read from sweep 2 on)
      const T* Zprev = zbuf(Z0, Z1, Z2, (s <= 2) ? src : (((s - 1) % 2 == 0) ? o1 : o2));
      stamp_wg(b, tm, s, 0);
      if constexpr (OPK == OP_FACTOR) {
        // first pass over the minibatch; in sweep 1 also the residuals and
        // the Gram matrix, from which the barrier's last arrival sets the shift
        const bool first = s == 1;
        factor_rows<T, KB, NT>(cfg.n, cfg.lda, cfg.m, cfg.batch, (const gbl<T>*)dstep.A, (const gbl<T>*)dstep.bq,
                               (const gbl<int>*)dstep.bidx, (const gbl<T>*)Zin, (gbl<T>*)dstep.qy,
                               (gbl<double>*)dstep.qw, (gbl<double>*)dstep.qn, (const gbl<Ctl>*)ctl, cfg.r, first,
                               (lds<char>*)xstage, tm.wg, tm.nwg);
        if (first)
          factor_gram<T, NT>(cfg.n, cfg.lda, cfg.m, cfg.batch, (const gbl<T>*)dstep.A, (const gbl<int>*)dstep.bidx,
                             (gbl<T>*)dstep.qk, (lds<T>*)xstage, tm.wg, tm.nwg);
        if (!grid_sync<NT>(b, tm, 0, [&] {
              if (first) {
                const double gmax =
                    factor_shift<T, NT>(cfg.n, cfg.batch, cfg.unit_round, (const gbl<T>*)dstep.qk,
                                        (const gbl<double>*)dstep.qw, (const gbl<double>*)dstep.qn,
                                        (lds<double>*)xstage);
                if (tid < 64) setup_step(cfg, (gbl<Ctl>*)ctl, gmax, tid);
              }
            }))
          return;
      }
      if constexpr (OPK == OP_CSR) {
        if (grad)
          apply_phase<T, KB, OPK, NT, true, CACHE>(cfg, ctl, dat, gvals, g, Bm, Zin, Zout, Zprev, b.part, smem, cc,
                                                   (lds<char>*)xstage, tm);
        else
          apply_phase<T, KB, OPK, NT, false, CACHE>(cfg, ctl, dat, gvals, g, Bm, Zin, Zout, Zprev, b.part, smem, cc,
                                                    (lds<char>*)xstage, tm);
      } else {
        apply_phase<T, KB, OPK, NT, false, false>(cfg, ctl, dstep, gvals, g, Bm, Zin, Zout, Zprev, b.part, smem, cc,
                                                  (lds<char>*)xstage, tm);
      }
      stamp_wg(b, tm, s, 1);
      int outcome = 0;
      if (!grid_sync<NT>(
              b, tm, PartRec<KB>::len(cfg.r, SM::XR != 0),
              [&]() -> int {
                stamp(b, 2 * s);
                gbl<Ctl>* gc = (gbl<Ctl>*)ctl;
                // every thread calls it (it runs on two wavefronts); with
                // kSweepEnded X_{t+1}, t + 1 and the scalars of step t + 1
                // are set.  Thread 0's value is the barrier's tag.
                int res = small_sweep<KB>((const lds<Cfg>*)&s_cfg, gc, (const lds<double>*)lsums,
                                          (lds<double>*)smem, s, in, out, grad, tid, (gbl<long long>*)b.ts);
                if ((res & kSweepEnded) && deadline != 0 && tid == 0 && (long long)wall_clock64() >= deadline) {
                  gc->pause_seq = seq;
                  res |= kSweepHalt;
                }
                stamp(b, 2 * s + 1);
                return res;
              },
              &outcome, lsums))
        return;
      if (outcome & kSweepHalt) return;  // failure, stopping rule or pause: ctl records which
      if (outcome & kSweepEnded) {
        src = (outcome & kSweepExtrap) ? out : in;
        break;
      }
    }
  }
}

template <typename T, int KB, int OPK, int NT, bool CACHE>
static __global__ __launch_bounds__(NT) void k_step(Cfg cfg, Ctl* __restrict__ ctl, Data<T> dat, T* __restrict__ Z0,
                                             T* __restrict__ Z1, T* __restrict__ Z2, T* __restrict__ g, Bufs b,
                                             int nsteps) {
  using L = StepLds<T, KB, OPK, NT>;
  __shared__ double smem[L::SMEM_DOUBLES];
  __shared__ __attribute__((aligned(16))) char xstage[L::XSTAGE_BYTES];
  extern __shared__ __attribute__((aligned(16))) char dyn[];  // CSR cache (CACHE)
  step_loop<T, KB, OPK, NT, CACHE>(cfg, ctl, dat, Z0, Z1, Z2, g, b, nsteps, grid_team(), smem, xstage, dyn);
}

// One resident instance of the batched step kernel.
template <typename T>
struct Slot {
  Cfg cfg;
  Ctl* ctl;
  Data<T> dat;
  T* Z0;
  T* Z1;
  T* Z2;
  Bufs b;      // its own partials, reduction buffers and barrier words
  int nwg;     // workgroups of its team
  int nsteps;  // iterations it runs in this launch (0: none)
};

// Batched persistent step kernel: the grid is split into teams, one per
// resident instance; team[w] = (slot, rank) of workgroup w (slot < 0: idle,
// the workgroup exits).  Every team runs until its instance's `nsteps` are
// done or the launch's time budget (wall-clock ticks, 0: none) is used up,
// whichever comes first; how steps fall into launches does not change an
// instance's arithmetic.  Each team runs its instance exactly as k_step does
// on a grid of nwg workgroups, with the instance's own barrier words and
// partials, so an instance's arithmetic (and its reduction order) does not
// depend on which other instances are resident.  Launched cooperatively.
// Per-launch parameters of k_serve, read from device memory so that a
// captured launch replays with new values: the launch number and its time
// budget in wall-clock ticks (0: none).
struct ServeParams {
  int64_t seq;
  long long budget;
};

template <typename T, int KB, int OPK, int NT>
static __global__ __launch_bounds__(NT) void k_serve(const Slot<T>* __restrict__ slots, const int2* __restrict__ team,
                                                     const ServeParams* __restrict__ prm) {
  using L = StepLds<T, KB, OPK, NT>;
  __shared__ double smem[L::SMEM_DOUBLES];
  __shared__ __attribute__((aligned(16))) char xstage[L::XSTAGE_BYTES];
  __shared__ long long s_t0;
  if (threadIdx.x == 0) s_t0 = (long long)wall_clock64();
  __syncthreads();
  const int64_t seq = prm->seq;
  const long long budget = prm->budget;
  const long long deadline = budget > 0 ? s_t0 + budget : 0;
  const int slot = __builtin_amdgcn_readfirstlane(team[blockIdx.x].x);
  const int rank = __builtin_amdgcn_readfirstlane(team[blockIdx.x].y);
  if (slot < 0) return;
  const Slot<T>* sl = slots + slot;
  const int nsteps = sl->nsteps;
  if (nsteps <= 0) return;
  const Cfg cfg = sl->cfg;
  const Data<T> dat = sl->dat;
  const Bufs b = sl->b;
  step_loop<T, KB, OPK, NT, false>(cfg, sl->ctl, dat, sl->Z0, sl->Z1, sl->Z2, nullptr, b, nsteps,
                                   Team{rank, sl->nwg}, smem, xstage, nullptr, deadline, seq);
}

// Orthonormalising transform of a freshly uploaded basis B = block `src`
// (cooperative launch with the step kernel's grid): Gram of B, then Wb = R^-1
// (B^T B = R^T R), so that Q = B Wb is orthonormal, and the step scalars.
template <typename T, int KB, int OPK, int NT>
static __global__ __launch_bounds__(NT) void k_basis(Cfg cfg, Ctl* __restrict__ ctl, T* __restrict__ Z0,
                                              T* __restrict__ Z1, T* __restrict__ Z2, Bufs b) {
  using SH = StepShape<T, KB, OPK, NT>;
  using SM = ApplySmem<T, KB, SH::ROWS, SH::GWROWS>;
  __shared__ double smem[SM::TOTAL];
  const int tid = threadIdx.x;
  const T* Bm = zbuf(Z0, Z1, Z2, ldi(&ctl->src));
  gram_phase<T, KB, SH::GROWS, NT>(cfg, (const gbl<T>*)Bm, (gbl<double>*)b.part, (lds<double>*)smem);
  grid_sync<NT>(b, grid_team(), KB * KB, [&] {
    if (tid < 64) {
      basis_setup<KB>(cfg, (gbl<Ctl>*)ctl, (const gbl<double>*)b.sums, (lds<double>*)smem, tid);
      wg_fence();
      step_scalars(cfg, (gbl<Ctl>*)ctl, tid);
    }
  });
}

// Q = B Wb written into the block after `src` (the next step's first output,
// so free between steps): the factored iterate's V = Q[:, :r] in explicit
// form, for the objective kernels.  One thread per element.
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_materialize(Cfg cfg, const Ctl* __restrict__ ctl, T* __restrict__ Z0,
                                                     T* __restrict__ Z1, T* __restrict__ Z2) {
  const int src = ctl->src;
  const T* Bm = zbuf(Z0, Z1, Z2, src);
  T* Q = zbuf(Z0, Z1, Z2, (src + 1) % 3);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cfg.n * KB; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / KB;
    const int c = (int)(e % KB);
    double z = 0.0;
#pragma unroll 8
    for (int q = 0; q < KB; ++q) z += (double)Bm[i * KB + q] * ctl->Wb[q * KB + c];
    Q[e] = (T)z;
  }
}

// sum over a 256-thread workgroup (fixed order); sred: 4 doubles of LDS
__device__ __forceinline__ double block_sum256(double v, double* sred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  return (sred[0] + sred[1]) + (sred[2] + sred[3]);
}

// ---------------------------------------------------------------------------
// Dual-averaging reading (MEG_FLAG_DUAL_AVERAGE): the log-domain matrix Y is
// kept dense and accumulated, Y_1 = log X_1, Y_{t+1} = Y_t - eta grad f(X_t);
// each step decomposes Y_{t+1} + sigma' I instead of M_t.  Q is the
// materialised basis (V = Q[:, :r]).
// ---------------------------------------------------------------------------
// Y = log X = log(alpha) I + V diag(c) V^T, one workgroup per row
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_da_init(Cfg cfg, const Ctl* __restrict__ ctl, const T* Z0,
                                                        const T* Z1, const T* Z2, T* __restrict__ Y) {
  __shared__ double vc[KMAX];
  const T* Q = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);
  const int64_t i = blockIdx.x, n = cfg.n;
  const int r = cfg.r;
  if (threadIdx.x < r) vc[threadIdx.x] = (double)Q[i * KB + threadIdx.x] * ctl->c[threadIdx.x];
  __syncthreads();
  const double la = log(ctl->alpha);
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    double y = (i == j) ? la : 0.0;
    for (int l = 0; l < r; ++l) y += vc[l] * (double)Q[j * KB + l];
    Y[i * n + j] = (T)y;
  }
  // lambda_min(log X) = log alpha (c >= 0)
  if (i == 0 && threadIdx.x == 0) ((Ctl*)ctl)->da_lmin = la;
}

// Y <- Y - eta G with G = C (linear) or X_t - M (denoising), one workgroup
// per row; part[i] = Y_ii - sum_{j != i} |Y_ij| of the new Y (Gershgorin)
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_da_update(Cfg cfg, const Ctl* __restrict__ ctl, const T* __restrict__ D,
                                                          const T* Z0, const T* Z1, const T* Z2, T* __restrict__ Y,
                                                          double* __restrict__ part) {
  __shared__ double vd[KMAX];
  const T* Q = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);
  __shared__ double sred[4];
  const int64_t i = blockIdx.x, n = cfg.n;
  const int r = cfg.r;
  const bool den = cfg.kind == DENOISE_DENSE;
  if (threadIdx.x < r) vd[threadIdx.x] = den ? (double)Q[i * KB + threadIdx.x] * ctl->d[threadIdx.x] : 0.0;
  __syncthreads();
  const double alpha = ctl->alpha, eta = cfg.eta;
  double off = 0.0, dia = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    double g = (double)D[i * cfg.ld + j];
    if (den) {
      double x = (i == j) ? alpha : 0.0;
      for (int l = 0; l < r; ++l) x += vd[l] * (double)Q[j * KB + l];
      g = x - g;
    }
    const T y = (T)((double)Y[i * n + j] - eta * g);
    Y[i * n + j] = y;
    if (i == j) dia = (double)y; else off += fabs((double)y);
  }
  off = block_sum256(off, sred);
  __syncthreads();
  dia = block_sum256(dia, sred);
  if (threadIdx.x == 0) part[i] = dia - off;
}

// the step's coefficients for Yhat = Y + sigma' I >= 0 (sigma' from the
// smallest Gershgorin bound): no low-rank term, the operator scale 1, and
// sigma = sigma' + log alpha so that the eigenvalues mu = theta + log alpha -
// sigma the step forms are those of Y; the first sweep's Chebyshev interval
// from the last step's mu_k.  One wavefront.
static __global__ __launch_bounds__(64) void k_da_setup(Cfg cfg, Ctl* __restrict__ ctl,
                                                        const double* __restrict__ part, int cnt) {
  const int lane = threadIdx.x;
  double m = __builtin_inf();
  for (int i = lane; i < cnt; i += 64) m = fmin(m, part[i]);
  m = wave_min(m);
  // Weyl: lambda_min(Y_{t+1}) >= lambda_min(Y_t) - eta lambda_max(grad f(X_t)),
  // with the objective's bound of lambda_max (the same as the step's shift
  // uses); the larger of the two lower bounds
  const double dl = (lane < cfg.r) ? ctl->d[lane] : 0.0;
  const double gmax = grad_bound(cfg, ctl->alpha, dl, ctl->op_lmin, ctl->op_lmax, 0, 0.0, 0.0, lane);
  m = fmax(m, ctl->da_lmin - cfg.eta * gmax);
  if (lane == 0) ctl->da_lmin = m;
  const double sp = -m + 1e-3 * (fabs(m) + 1.0);
  if (lane < KMAX) ctl->ceff[lane] = 0.0;
  if (lane == 0) {
    const double la = log(ctl->alpha);
    ctl->gmax = 0.0;
    ctl->sigma = sp + la;
    ctl->sdiag = sp;
    ctl->opscale = 1.0;
    double b = 0.0;
    if (cfg.cheb && ctl->mu_valid) {
      const double bk = ctl->mu_k + sp, b1 = ctl->mu_1 + sp;
      if (bk > 1e-3 * b1 && bk < 0.5 * b1) b = bk;
    }
    ctl->cheb_b = b;
  }
}

// ---------------------------------------------------------------------------
// auxiliary kernels (ordinary launches; per-workgroup partials, then k_finish)
// ---------------------------------------------------------------------------
// A dense operand in the state's type, or as bf16 planes hi + lo (their sum,
// exact in FP64, is the matrix the matrix-core apply multiplies by).
template <typename T>
struct DenseSrc {
  const T* D;
  const uint16_t* hi;
  const uint16_t* lo;
  __device__ __forceinline__ double at(int64_t idx) const {
    return hi ? (double)bf16_val(hi[idx]) + (double)bf16_val(lo[idx]) : (double)D[idx];
  }
};

// objective at X_t, dense kinds: LINEAR sum C_ij X_ij, DENOISE 1/2 sum (X_ij - M_ij)^2
// X_ij = alpha [i == j] + sum_l V_il d_l V_jl, accumulated in FP64; one wave
// per row; V from k_materialize
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_objective_dense(Cfg cfg, const Ctl* __restrict__ ctl,
                                                         DenseSrc<T> D, const T* __restrict__ Z0,
                                                         const T* __restrict__ Z1, const T* __restrict__ Z2,
                                                         double* __restrict__ part) {
  const T* Qw = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);  // written by k_materialize
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
      const double dij = D.at(i * cfg.ld + j);
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
static __global__ __launch_bounds__(256) void k_objective_csr(Cfg cfg, const Ctl* __restrict__ ctl, const int* __restrict__ rp,
                                                       const int* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ Z0, const T* __restrict__ Z1,
                                                       const T* __restrict__ Z2, double* __restrict__ part) {
  const T* Qw = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);  // written by k_materialize
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

// <X_t, G_t> for the dual gap (Section 7), G_t = grad f(X_t), accumulated in
// FP64 like the objective: LINEAR sum C_ij X_ij; DENOISE sum X_ij (X_ij - M_ij).
// One wave per row; V from k_materialize.
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_xdotg_dense(Cfg cfg, const Ctl* __restrict__ ctl, DenseSrc<T> D,
                                                            const T* __restrict__ Z0, const T* __restrict__ Z1,
                                                            const T* __restrict__ Z2, double* __restrict__ part) {
  const T* Qw = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);
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
      const double dij = D.at(i * cfg.ld + j);
      acc += (cfg.kind == LINEAR_DENSE) ? dij * x : x * (x - dij);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) sred[wave] = acc;
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// <X_t, G_t> on the pattern: LINEAR sum_Omega C_ij X_ij; MASKED
// sum_Omega X_ij (X_ij - M_ij), with the gradient values X_ij - M_ij also
// written to gout (the operator the dual gap's Lanczos run multiplies by).
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_xdotg_csr(Cfg cfg, const Ctl* __restrict__ ctl,
                                                          const int* __restrict__ rp, const int* __restrict__ col,
                                                          const T* __restrict__ val, T* __restrict__ gout,
                                                          const T* __restrict__ Z0, const T* __restrict__ Z1,
                                                          const T* __restrict__ Z2, double* __restrict__ part) {
  const T* Qw = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);
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
      if (cfg.kind == LINEAR_CSR) {
        acc += v * x;
      } else {
        acc += x * (x - v);
        gout[e] = (T)(x - v);
      }
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) sred[wave] = acc;
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// sum of squares of a strided matrix (rows x cols, ld) or a vector (rows = 1)
template <typename T>
static __global__ __launch_bounds__(256) void k_sumsq(DenseSrc<T> x, int64_t rows, int64_t cols, int64_t ld,
                                               double* __restrict__ part) {
  __shared__ double sred[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc = 0.0;
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e % cols;
    const double v = x.at(i * ld + j);
    acc += v * v;
  }
  acc = wave_sum(acc);
  if (lane == 0) sred[wave] = acc;
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// Sum nwg partials in a fixed order and store: what = 0 -> f (objective),
// 1 -> data_norm = sqrt(sum).  One workgroup.
static __global__ __launch_bounds__(256) void k_finish(Ctl* __restrict__ ctl, const double* __restrict__ part, int nwg,
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
// Used by the Lanczos estimate of the data operator's extreme eigenvalues
// (once per context) and by the dual gap's Lanczos run for lambda_min of the
// gradient (there with the gradient values as the CSR values).  One wave per
// row.
template <typename T>
static __global__ __launch_bounds__(256) void k_matvec(Cfg cfg, DenseSrc<T> D, const int* __restrict__ rp,
                                                const int* __restrict__ col, const T* __restrict__ val,
                                                const T* __restrict__ x, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= cfg.n) return;
  double acc = 0.0;
  if (cfg.kind == LINEAR_DENSE || cfg.kind == DENOISE_DENSE) {
    for (int64_t j = lane; j < cfg.n; j += 64) acc += D.at(i * cfg.ld + j) * (double)x[j];
  } else {
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) acc += (double)val[e] * (double)x[col[e]];
  }
  acc = wave_sum(acc);
  if (lane == 0) y[i] = acc;
}

// ---------------------------------------------------------------------------
// Lanczos vectors of the dual gap's lambda_min run, all in FP64 on the device
// (V: the basis, row l = vector l of length n).  Reductions are per workgroup
// (256 threads) in a fixed order.
// ---------------------------------------------------------------------------

// out[l] = V[l] . w for l < cnt: one workgroup per vector
static __global__ __launch_bounds__(256) void k_lz_dots(const double* __restrict__ V, const double* __restrict__ w,
                                                        int64_t n, double* __restrict__ out) {
  __shared__ double sred[4];
  const double* v = V + (int64_t)blockIdx.x * n;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) a += v[i] * w[i];
  a = block_sum256(a, sred);
  if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// w -= sum_{l < cnt} h[l] V[l]  (one reorthogonalisation pass)
static __global__ __launch_bounds__(256) void k_lz_sub(const double* __restrict__ V, const double* __restrict__ h,
                                                       int cnt, int64_t n, double* __restrict__ w) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int l = 0; l < cnt; ++l) s += h[l] * V[(int64_t)l * n + i];
    w[i] -= s;
  }
}

// u = sum_{l < cnt} s[l] V[l]  (a Ritz vector from the basis)
static __global__ __launch_bounds__(256) void k_lz_combine(const double* __restrict__ V, const double* __restrict__ s,
                                                           int cnt, int64_t n, double* __restrict__ u) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double a = 0.0;
    for (int l = 0; l < cnt; ++l) a += s[l] * V[(int64_t)l * n + i];
    u[i] = a;
  }
}

// x (the product's input, in the state's type) = (T) V[j]
template <typename T>
static __global__ __launch_bounds__(256) void k_lz_cast(const double* __restrict__ v, int64_t n, T* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = (T)v[i];
}

// denoising gradient G = alpha I + V diag(d) V^T - M: p[l] = sum_i Q[i][l] x[i]
// for the first r columns of the materialised basis Q (row stride KB), one
// workgroup per column
template <typename T>
static __global__ __launch_bounds__(256) void k_lz_lr_dots(const T* __restrict__ Q, int KB, const T* __restrict__ x,
                                                           int64_t n, double* __restrict__ p) {
  __shared__ double sred[4];
  const int l = blockIdx.x;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) a += (double)Q[i * KB + l] * (double)x[i];
  a = block_sum256(a, sred);
  if (threadIdx.x == 0) p[l] = a;
}
// y <- alpha x + sum_l Q[i][l] d_l p[l] - y   (y held M x)
template <typename T>
static __global__ __launch_bounds__(256) void k_lz_lr_update(const Ctl* __restrict__ ctl, const T* __restrict__ Q, int KB,
                                                             int r, const T* __restrict__ x,
                                                             const double* __restrict__ p, int64_t n,
                                                             double* __restrict__ y) {
  const double alpha = ctl->alpha;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double s = alpha * (double)x[i] - y[i];
    for (int l = 0; l < r; ++l) s += (double)Q[i * KB + l] * ctl->d[l] * p[l];
    y[i] = s;
  }
}

// deflation by the first r columns of the materialised basis Q (row stride
// KB): p[l] = sum_i Q[i][l] w[i], one workgroup per column ...
template <typename T>
static __global__ __launch_bounds__(256) void k_lz_defl_dots(const T* __restrict__ Q, int KB,
                                                             const double* __restrict__ w, int64_t n,
                                                             double* __restrict__ p) {
  __shared__ double sred[4];
  const int l = blockIdx.x;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) a += (double)Q[i * KB + l] * w[i];
  a = block_sum256(a, sred);
  if (threadIdx.x == 0) p[l] = a;
}
// ... then w -= Q[:, :r] p
template <typename T>
static __global__ __launch_bounds__(256) void k_lz_defl_sub(const T* __restrict__ Q, int KB, int r,
                                                            const double* __restrict__ p, int64_t n,
                                                            double* __restrict__ w) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int l = 0; l < r; ++l) s += (double)Q[i * KB + l] * p[l];
    w[i] -= s;
  }
}

// v = w / ||w|| (one workgroup): the start vector after its deflation
static __global__ __launch_bounds__(256) void k_lz_unit(const double* __restrict__ w, int64_t n,
                                                        double* __restrict__ v) {
  __shared__ double sred[4];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) a += w[i] * w[i];
  const double b = sqrt(block_sum256(a, sred));
  const double ib = b > 0.0 ? 1.0 / b : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) v[i] = w[i] * ib;
}

// w = y - alpha_j v_j - beta_{j-1} v_{j-1}, with alpha_j = ab[j] (from
// k_lz_dots of v_j and y) and beta_{j-1} = ab[m + j - 1]
static __global__ __launch_bounds__(256) void k_lz_three_term(const double* __restrict__ V, const double* __restrict__ y,
                                                              const double* __restrict__ ab, int j, int m, int64_t n,
                                                              double* __restrict__ w) {
  const double a = ab[j], b = j > 0 ? ab[m + j - 1] : 0.0;
  const double* v = V + (int64_t)j * n;
  const double* vp = V + (int64_t)(j > 0 ? j - 1 : 0) * n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    w[i] = y[i] - a * v[i] - b * vp[i];
}

// beta_j = ||w|| into ab[m + j]; v_{j+1} = w / beta_j, or zero once the
// Krylov space is invariant (beta_j <= 1e-14 |alpha_j|): one workgroup
static __global__ __launch_bounds__(256) void k_lz_next(const double* __restrict__ w, int j, int m, int64_t n,
                                                        double* __restrict__ ab, double* __restrict__ V) {
  __shared__ double sred[4];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) a += w[i] * w[i];
  const double b = sqrt(block_sum256(a, sred));
  const bool live = b > 1e-14 * (fabs(ab[j]) + 1e-300);
  if (threadIdx.x == 0) ab[m + j] = live ? b : 0.0;
  double* vn = V + (int64_t)(j + 1) * n;
  const double ib = live ? 1.0 / b : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) vn[i] = w[i] * ib;
}

// ---------------------------------------------------------------------------
// Batched Lanczos runs of the full-trace estimate: up to 64 vectors advance
// in lockstep, stored interleaved (element (i, b) at i * 64 + b), so lane b of
// a wave owns vector b and one read of an operator row serves all of them.
// Reductions over rows are per workgroup in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kTrW = 64;

// Y = Op X for a CSR operator (values: C, M or the gradient values on the
// pattern): one wave per row, lane = vector.  The row's column indices and
// values are read 64 at a time (lane j holds entry j) and broadcast with
// readlane, so the loads of the X rows they select do not wait on each other.
template <typename T>
static __global__ __launch_bounds__(256) void k_tr_matvec_csr(int64_t n, const int* __restrict__ rp,
                                                              const int* __restrict__ col, const T* __restrict__ val,
                                                              const double* __restrict__ X, double* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int e1 = rp[i + 1];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int e0 = rp[i]; e0 < e1; e0 += 64) {
    const int cnt = min(64, e1 - e0);
    // entries past the row's end select row 0 with weight 0
    const int cj = lane < cnt ? col[e0 + lane] : 0;
    const double vj = lane < cnt ? (double)val[e0 + lane] : 0.0;
    for (int j = 0; j < cnt; j += 4) {
      const int c0 = __builtin_amdgcn_readlane(cj, j), c1 = __builtin_amdgcn_readlane(cj, j + 1);
      const int c2 = __builtin_amdgcn_readlane(cj, j + 2), c3 = __builtin_amdgcn_readlane(cj, j + 3);
      const double x0 = X[(int64_t)c0 * kTrW + lane], x1 = X[(int64_t)c1 * kTrW + lane];
      const double x2 = X[(int64_t)c2 * kTrW + lane], x3 = X[(int64_t)c3 * kTrW + lane];
      a0 += readlane_d(vj, j) * x0;
      a1 += readlane_d(vj, j + 1) * x1;
      a2 += readlane_d(vj, j + 2) * x2;
      a3 += readlane_d(vj, j + 3) * x3;
    }
  }
  Y[i * kTrW + lane] = (a0 + a1) + (a2 + a3);
}

// Y = D X for a dense operator (n x n, stride ld; the state's type or bf16
// planes): a workgroup computes 32 rows x 64 vectors, staging 32-column
// chunks of D and the matching 32 rows of X in LDS (FP64); a thread holds
// 2 rows x 4 vectors.
template <typename T>
static __global__ __launch_bounds__(256) void k_tr_matvec_dense(int64_t n, int64_t ld, DenseSrc<T> D,
                                                                const double* __restrict__ X,
                                                                double* __restrict__ Y) {
  __shared__ double Ds[32][33];
  __shared__ double Xs[32][kTrW];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const int64_t row0 = (int64_t)blockIdx.x * 32;
  double acc[2][4] = {};
  for (int64_t k0 = 0; k0 < n; k0 += 32) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int e = tid + 256 * s, rr = e >> 5, kk = e & 31;
      const int64_t gi = row0 + rr, gk = k0 + kk;
      Ds[rr][kk] = (gi < n && gk < n) ? D.at(gi * ld + gk) : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int e = tid + 256 * s, kk = e >> 6, b = e & 63;
      const int64_t gk = k0 + kk;
      Xs[kk][b] = gk < n ? X[gk * kTrW + b] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      const double d0 = Ds[2 * ty][kk], d1 = Ds[2 * ty + 1][kk];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double x = Xs[kk][tx + 16 * q];
        acc[0][q] += d0 * x;
        acc[1][q] += d1 * x;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int64_t gi = row0 + 2 * ty + a;
    if (gi < n) {
#pragma unroll
      for (int q = 0; q < 4; ++q) Y[gi * kTrW + tx + 16 * q] = acc[a][q];
    }
  }
}

// Column dot products, in two passes for a fixed summation order: workgroup
// g of the partial kernels takes rows g*4 + w + 4*G*q (w its wave, lane = the
// vector) and writes one partial per output; k_tr_part_sum adds the G
// partials of each output in order.  kTrRedWG bounds G.
constexpr int kTrRedWG = 256;

// part[(g * na + l) * 64 + b] = sum over workgroup g's rows i of
// A[i * lda + l] X[i * 64 + b], l < na <= 32 (A: the state's basis, or the
// interleaved FP64 deflation basis)
template <typename TA>
static __global__ __launch_bounds__(256) void k_tr_gram_part(const TA* __restrict__ A, int64_t lda, int na,
                                                             const double* __restrict__ X, int64_t n,
                                                             double* __restrict__ part) {
  __shared__ double s[4][kTrW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc[32];
#pragma unroll
  for (int l = 0; l < 32; ++l) acc[l] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < n; i += (int64_t)gridDim.x * 4) {
    const double x = X[i * kTrW + lane];
    const TA* a = A + i * lda;
#pragma unroll
    for (int l = 0; l < 32; ++l)
      if (l < na) acc[l] += (double)a[l] * x;
  }
#pragma unroll
  for (int l = 0; l < 32; ++l) {
    if (l >= na) break;
    s[w][lane] = acc[l];
    __syncthreads();
    if (w == 0) part[((int64_t)blockIdx.x * na + l) * kTrW + lane] = (s[0][lane] + s[1][lane]) + (s[2][lane] + s[3][lane]);
    __syncthreads();
  }
}

// part[g * 64 + b] = sum over workgroup g's rows i of A[i][b] B[i][b]
static __global__ __launch_bounds__(256) void k_tr_cdot_part(const double* __restrict__ A,
                                                             const double* __restrict__ B, int64_t n,
                                                             double* __restrict__ part) {
  __shared__ double s[4][kTrW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a0 = 0.0, a1 = 0.0;
  int64_t i = (int64_t)blockIdx.x * 4 + w;
  const int64_t st = (int64_t)gridDim.x * 4;
  for (; i + st < n; i += 2 * st) {
    a0 += A[i * kTrW + lane] * B[i * kTrW + lane];
    a1 += A[(i + st) * kTrW + lane] * B[(i + st) * kTrW + lane];
  }
  if (i < n) a0 += A[i * kTrW + lane] * B[i * kTrW + lane];
  s[w][lane] = a0 + a1;
  __syncthreads();
  if (w == 0) part[(int64_t)blockIdx.x * kTrW + lane] = (s[0][lane] + s[1][lane]) + (s[2][lane] + s[3][lane]);
}

// out[o] = sum_{g < G} part[g * cnt + o] for o < cnt (cnt = na * 64): one
// wave per output, lane j adding partials j, j + 64, ... in order, then the
// wave's fixed-order reduction
static __global__ __launch_bounds__(256) void k_tr_part_sum(const double* __restrict__ part, int G, int cnt,
                                                            double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= cnt) return;
  double a = 0.0;
  for (int g = lane; g < G; g += 64) a += part[(int64_t)g * cnt + o];
  a = wave_sum(a);
  if (lane == 0) out[o] = a;
}

// Y[i][b] = s Y[i][b] + c0 X[i][b] + sum_{l < r} Q[i][l] cv[l] P[l][b]: with
// Y = Op X on entry this makes Y = M_t X (the data term, the identity term and
// the low-rank term of log X_t; P from the column dots of the basis).
template <typename T>
static __global__ __launch_bounds__(256) void k_tr_opfix(const T* __restrict__ Q, int KB, int r,
                                                         const double* __restrict__ cv,
                                                         const double* __restrict__ P, double s, double c0,
                                                         const double* __restrict__ X, int64_t n,
                                                         double* __restrict__ Y) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * kTrW; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e >> 6;
    const int b = (int)(e & 63);
    double a = s * Y[e] + c0 * X[e];
    for (int l = 0; l < r; ++l) a += (double)Q[i * KB + l] * cv[l] * P[l * kTrW + b];
    Y[e] = a;
  }
}

// W = Y - alpha_b X - beta_b Xp with alpha_b = al[b] and beta_b = be[b] (the
// previous step's beta; be = nullptr at the first step)
static __global__ __launch_bounds__(256) void k_tr_three(const double* __restrict__ Y, const double* __restrict__ X,
                                                         const double* __restrict__ Xp,
                                                         const double* __restrict__ al,
                                                         const double* __restrict__ be, int64_t n,
                                                         double* __restrict__ W) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * kTrW; e += (int64_t)gridDim.x * 256) {
    const int b = (int)(e & 63);
    double w = Y[e] - al[b] * X[e];
    if (be) w -= be[b] * Xp[e];
    W[e] = w;
  }
}

// beta_b = sqrt(bsq[b]) (zero once vector b's Krylov space is invariant:
// beta_b <= 1e-14 (|alpha_b| + |beta_prev_b|), or the vector is zero); be[b]
// receives beta_b, and W becomes the next Lanczos vector W / beta_b
static __global__ __launch_bounds__(256) void k_tr_next(const double* __restrict__ bsq,
                                                        const double* __restrict__ al,
                                                        const double* __restrict__ bprev, int64_t n,
                                                        double* __restrict__ be, double* __restrict__ W) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * kTrW; e += (int64_t)gridDim.x * 256) {
    const int b = (int)(e & 63);
    const double bt = sqrt(fmax(bsq[b], 0.0));
    const double ref = fabs(al[b]) + (bprev ? fabs(bprev[b]) : 0.0);
    const bool live = bt > 1e-14 * ref && bt > 1e-300;
    if (e < kTrW) be[b] = live ? bt : 0.0;
    W[e] = live ? W[e] / bt : 0.0;
  }
}

// Start block: columns [0, kq) from the FP64 interleaved basis Qd or, when Qd
// is null, from the state's basis Q (n x KB, the state's type); columns
// [kq, kq + np) from probes (n x np column-major FP64, probe j at
// probes + j * n); the rest zero.
template <typename T>
static __global__ __launch_bounds__(256) void k_tr_load(const T* __restrict__ Q, int KB,
                                                        const double* __restrict__ Qd, int kq,
                                                        const double* __restrict__ probes, int np, int64_t n,
                                                        double* __restrict__ X) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * kTrW; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e >> 6;
    const int b = (int)(e & 63);
    double v = 0.0;
    if (b < kq) v = Qd ? Qd[e] : (double)Q[i * KB + b];
    else if (b < kq + np) v = probes[(int64_t)(b - kq) * n + i];
    X[e] = v;
  }
}

// Row mix: Y[i][b] = (sub ? Y[i][b] - s : s) for b in [b0, b1), with
// s = sum_{l < nl} A[i][l] Mx[l][b] (Mx row-major 64 x 64).  A and Y may be the
// same buffer: a wave reads its row whole before it writes.  One wave per row.
static __global__ __launch_bounds__(256) void k_tr_rowmix(const double* A, const double* __restrict__ Mx, int nl,
                                                          int b0, int b1, int sub, int64_t n, double* Y) {
  __shared__ double Ms[kTrW * kTrW];
  for (int e = threadIdx.x; e < nl * kTrW; e += 256) Ms[e] = Mx[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double a = A[i * kTrW + lane];
  const double y = Y[i * kTrW + lane];
  double s = 0.0;
  for (int l = 0; l < nl; ++l) s += __shfl(a, l) * Ms[l * kTrW + lane];
  if (lane >= b0 && lane < b1) Y[i * kTrW + lane] = sub ? y - s : s;
}

// X[i][b] *= sc[b]
static __global__ __launch_bounds__(256) void k_tr_scale(const double* __restrict__ sc, int64_t n,
                                                         double* __restrict__ X) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * kTrW; e += (int64_t)gridDim.x * 256)
    X[e] *= sc[e & 63];
}

// ---------------------------------------------------------------------------
// Bilinear measurements f(X) = 1/2 sum_i (tr(A_i^T X B_i) - y_i)^2 (the
// recovery problem of the experiments; rank-1 measurements a_i^T X b_i for
// p = 1): residuals at the factored iterate, then the dense symmetric gradient
// 1/2 sum_i r_i (A_i B_i^T + B_i A_i^T).  A holds 2mp rows of length lda: row
// i p + q is column q of A_i, row m p + i p + q column q of B_i.
// ---------------------------------------------------------------------------
// r_i = sum_q [alpha a_iq^T b_iq + sum_{l < r} d_l (a_iq^T v_l)(b_iq^T v_l)] - y_i with V the
// first r columns of the basis k_materialize wrote (n x KB): one wave per
// measurement, FP64 sums; part[blockIdx.x] = 1/2 sum of r_i^2 over the
// workgroup's measurements.
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_bil_resid(Cfg cfg, const Ctl* __restrict__ ctl, const T* Z0,
                                                          const T* Z1, const T* Z2, const T* __restrict__ A,
                                                          int64_t lda, const T* __restrict__ y, int64_t m, int p,
                                                          double* __restrict__ res, double* __restrict__ part,
                                                          int qlds) {
  const T* Q = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);  // written by k_materialize
  __shared__ double sred[4];
  // qlds: V (the r used columns of Q) staged transposed in dynamic LDS,
  // Vt[l n + j] = Q[j][l], so a wave's reads of V_l are contiguous (Q's rows
  // are KB wide: reading Q[j][l] across lanes strides by a row)
  extern __shared__ __attribute__((aligned(16))) char dyn[];
  T* Vt = reinterpret_cast<T*>(dyn);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = cfg.r;
  const int64_t n = cfg.n;
  if (qlds) {
    for (int64_t e = threadIdx.x; e < (int64_t)r * n; e += 256) Vt[e] = Q[(e % n) * KB + e / n];
    __syncthreads();
  }
  double fsum = 0.0;
  const int64_t mp = m * p;
  // the contribution of one column pair: alpha a^T b + sum_l d_l (a^T v_l)(b^T v_l)
  auto pair_term = [&](const T* a, const T* b) -> double {
    double pa[KB], pb[KB], ab = 0.0;
#pragma unroll
    for (int l = 0; l < KB; ++l) pa[l] = pb[l] = 0.0;
    // columns in chunks of 8 x 64: the chunk's loads are issued together,
    // then its sums (the same per-lane order as one column at a time)
    constexpr int CH = 8;
    for (int64_t j0 = lane; j0 < n; j0 += 64 * CH) {
      T av[CH], bv[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int64_t j = j0 + 64 * u;
        av[u] = j < n ? a[j] : (T)0;
        bv[u] = j < n ? b[j] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int64_t j = j0 + 64 * u;
        if (j < n) {
          const double aj = (double)av[u], bj = (double)bv[u];
          ab += aj * bj;
          const T* q = Q + j * KB;
#pragma unroll
          for (int l = 0; l < KB; ++l) {
            if (l < r) {
              const double v = (double)(qlds ? Vt[l * n + j] : q[l]);
              pa[l] += aj * v;
              pb[l] += bj * v;
            }
          }
        }
      }
    }
    double t = ctl->alpha * wave_sum(ab);
#pragma unroll
    for (int l = 0; l < KB; ++l)
      if (l < r) t += ctl->d[l] * wave_sum(pa[l]) * wave_sum(pb[l]);
    return t;
  };
  for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < m; i += (int64_t)gridDim.x * 4) {
    double s = 0.0;
    if (p == 1) {
      s = pair_term(A + i * lda, A + (m + i) * lda);
    } else {
      for (int qc = 0; qc < p; ++qc) s += pair_term(A + (i * p + qc) * lda, A + (mp + i * p + qc) * lda);
    }
    const double ri = s - (double)y[i];
    if (lane == 0) res[i] = ri;
    fsum += 0.5 * ri * ri;
  }
  if (lane == 0) sred[wave] = fsum;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sred[0] + sred[1]) + (sred[2] + sred[3]);
}

// Partial gradients over the upper triangle of 64 x 64 tiles: workgroup x
// takes the tile pair (J, K), J <= K, of its index, slice s = blockIdx.z of
// the R = mp measurement rows; P_s[J,K][jl][kl] = sum_{rows i in slice s}
// r_{i/p} (a_ij b_ik + b_ij a_ik) with j = 64 J + jl, k = 64 K + kl.  A dense
// contraction over the rows, on the FP64 matrix cores: rows are staged 16 at a
// time in LDS (the J side scaled by the residual as it is read), each wave owns a 32 x 32
// quarter of the tile as 2 x 2 blocks of 16 x 16, and every 4-row step issues
// v_mfma_f64_16x16x4f64 twice per block (r a_J with b_K, r b_J with a_K).
// Operand layout: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// result register v of lane l is C[l / 16 + 4 v][l % 16].
constexpr int kBilTile = 64;

__device__ inline void bil_pair(int pair, int T, int& J, int& K) {
  J = 0;
  while (pair >= T - J) {
    pair -= T - J;
    ++J;
  }
  K = J + pair;
}

template <typename T>
static __global__ __launch_bounds__(256) void k_bil_grad_part(int64_t n, const T* __restrict__ A, int64_t lda,
                                                              int64_t m, int p, const double* __restrict__ res,
                                                              int64_t per_slice, int tiles,
                                                              double* __restrict__ P) {
  // Rows staged in the state's type, double-buffered: the next 16 rows are
  // loaded into registers before this stage's matrix-core work and stored to
  // the other buffer after it, so their latency overlaps the products; one
  // barrier per stage.  The J side is scaled by the residual as it is read
  // (the same FP64 product r_i a_ij as staging it scaled).
  __shared__ T sJa[2][16][kBilTile], sJb[2][16][kBilTile], sKa[2][16][kBilTile], sKb[2][16][kBilTile];
  __shared__ double sr[2][16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int jw = 32 * (wave >> 1), kw = 32 * (wave & 1);  // the wave's quarter of the tile
  const int li = lane & 15, lk = lane >> 4;
  int J, K;
  bil_pair(blockIdx.x, tiles, J, K);
  const int64_t j0 = (int64_t)J * kBilTile, k0 = (int64_t)K * kBilTile;
  const int64_t i_beg = (int64_t)blockIdx.z * per_slice;
  const int64_t i_end = min(m, i_beg + per_slice);
  f64x4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  // thread tid stages column jj = tid % 64 of rows ii = tid / 64 + 4 s
  const int jj = tid & 63, ib = tid >> 6;
  const bool okj = j0 + jj < n, okk = k0 + jj < n;
  T va[4], vb[4], wa[4], wb[4];
  double rv[4];
  auto gload = [&](int64_t i0) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int64_t i = i0 + ib + 4 * s4;
      const bool ok = i < i_end;
      rv[s4] = ok ? res[i / p] : 0.0;
      va[s4] = ok && okj ? A[i * lda + j0 + jj] : (T)0;
      vb[s4] = ok && okj ? A[(m + i) * lda + j0 + jj] : (T)0;
      wa[s4] = ok && okk ? A[i * lda + k0 + jj] : (T)0;
      wb[s4] = ok && okk ? A[(m + i) * lda + k0 + jj] : (T)0;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int ii = ib + 4 * s4;
      sJa[buf][ii][jj] = va[s4];
      sJb[buf][ii][jj] = vb[s4];
      sKa[buf][ii][jj] = wa[s4];
      sKb[buf][ii][jj] = wb[s4];
      if (jj == 0) sr[buf][ii] = rv[s4];
    }
  };
  if (i_beg < i_end) {
    gload(i_beg);
    lstore(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t i0 = i_beg; i0 < i_end; i0 += 16, buf ^= 1) {
    const bool more = i0 + 16 < i_end;
    if (more) gload(i0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = 4 * ks + lk;
      const double rk = sr[buf][kk];
      double xa[2], xb[2], ya[2], yb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        xa[t] = rk * (double)sJa[buf][kk][jw + 16 * t + li];
        xb[t] = rk * (double)sJb[buf][kk][jw + 16 * t + li];
        ya[t] = (double)sKa[buf][kk][kw + 16 * t + li];
        yb[t] = (double)sKb[buf][kk][kw + 16 * t + li];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], yb[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[a], ya[b], acc[a][b], 0, 0, 0);
        }
    }
    // the other buffer was last read in the previous stage, before the
    // barrier that ended it
    if (more) lstore(buf ^ 1);
    __syncthreads();
  }
  double* dst = P + ((int64_t)blockIdx.z * gridDim.x + blockIdx.x) * (kBilTile * kBilTile);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        dst[(jw + 16 * a + lk + 4 * v) * kBilTile + kw + 16 * b + li] = acc[a][b][v];
}

// G[j][k] = G[k][j] = 1/2 sum_{s < S} P_s[J,K][jl][kl] in slice order, in the
// state's type; diagonal tiles take their upper triangle, so G is exactly
// symmetric
template <typename T>
static __global__ __launch_bounds__(256) void k_bil_grad_sum(int64_t n, int S, int pairs, int tiles,
                                                             const double* __restrict__ P, T* __restrict__ G) {
  const int64_t per = (int64_t)kBilTile * kBilTile;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)pairs * per;
       e += (int64_t)gridDim.x * 256) {
    const int pair = (int)(e / per);
    const int w = (int)(e % per), jl = w / kBilTile, kl = w % kBilTile;
    int J, K;
    bil_pair(pair, tiles, J, K);
    const int64_t j = (int64_t)J * kBilTile + jl, k = (int64_t)K * kBilTile + kl;
    if (j >= n || k >= n || (J == K && jl > kl)) continue;
    double a = 0.0;
    for (int s = 0; s < S; ++s) a += P[((int64_t)s * pairs + pair) * per + w];
    const T v = (T)(0.5 * a);
    G[j * n + k] = v;
    G[k * n + j] = v;
  }
}

// CSR structure check: 0 = rp[0] <= rp[i] <= rp[i+1] <= rp[n] = nnz and every
// column index in [0, n).  Row ranges are validated before col is read.
// objective at X_t, quadratic measurements: 1/(2m) sum_i (a_i^T X a_i - b_i)^2
// over the whole pool, a_i^T X a_i = alpha ||a_i||^2 + sum_l d_l (a_i^T v_l)^2.
// Each wave takes MB measurements at a time so that a row of V read once
// serves all of them; lane partials in the state's type, reductions in FP64.
template <typename T, int KB>
static __global__ __launch_bounds__(256) void k_objective_quad(Cfg cfg, const Ctl* __restrict__ ctl, const T* __restrict__ A,
                                                        const T* __restrict__ bq, const T* __restrict__ Z0,
                                                        const T* __restrict__ Z1, const T* __restrict__ Z2,
                                                        double* __restrict__ part) {
  constexpr int MB = sizeof(T) == 4 ? 4 : 2;
  const T* Qw = zbuf(Z0, Z1, Z2, (ctl->src + 1) % 3);  // written by k_materialize
  __shared__ double sd[KMAX];
  __shared__ double sred[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = cfg.r;
  if (tid < KMAX) sd[tid] = ctl->d[tid];
  __syncthreads();
  const double alpha = ctl->alpha;
  double acc = 0.0;
  for (int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * MB; i0 < cfg.m; i0 += (int64_t)gridDim.x * 4 * MB) {
    T p[MB][KB], sa[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      sa[u] = 0;
#pragma unroll
      for (int l = 0; l < KB; ++l) p[u][l] = 0;
    }
    for (int64_t j = lane; j < cfg.n; j += 64) {
      T v[KB];
#pragma unroll
      for (int l = 0; l < KB; ++l) v[l] = (l < r) ? Qw[j * KB + l] : (T)0;
#pragma unroll
      for (int u = 0; u < MB; ++u) {
        const int64_t i = (i0 + u < cfg.m) ? i0 + u : cfg.m - 1;
        const T a = A[i * cfg.lda + j];
        sa[u] += a * a;
#pragma unroll
        for (int l = 0; l < KB; ++l) p[u][l] += a * v[l];
      }
    }
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      double x = alpha * wave_sum((double)sa[u]);
#pragma unroll
      for (int l = 0; l < KB; ++l)
        if (l < r) {
          const double q = wave_sum((double)p[u][l]);
          x += sd[l] * q * q;
        }
      if (i0 + u < cfg.m) {
        const double res = x - (double)bq[i0 + u];
        acc += 0.5 * res * res / (double)cfg.m;
      }
    }
  }
  if (lane == 0) sred[wave] = acc;  // identical in every lane
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// ---------------------------------------------------------------------------
// admission kernels of the batched server
// ---------------------------------------------------------------------------
// bf16 planes of an FP32 matrix: hi = RNE(x), lo = RNE(x - hi); columns n..ld-1 zero
static __global__ __launch_bounds__(256) void k_split_bf16(const float* __restrict__ M, int64_t ldm, int64_t n,
                                                    uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                                    int64_t ld) {
  const int64_t total = n * ld;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / ld, j = e % ld;
    const float x = (j < n) ? M[i * ldm + j] : 0.0f;
    const unsigned short h = bf16_rne(x);
    hi[e] = h;
    lo[e] = bf16_rne(x - bf16_val(h));
  }
}

// Gershgorin bounds of the planes' matrix hi + lo: per workgroup the min of
// a_ii - sum_{j != i} |a_ij| and the max of a_ii + sum_{j != i} |a_ij| over
// its rows (one wave per row, FP64 sums) -> part[2 wg], part[2 wg + 1]
static __global__ __launch_bounds__(256) void k_gersh(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo,
                                               int64_t n, int64_t ld, double* __restrict__ part) {
  __shared__ double sl[4], sh[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double lmin = __builtin_inf(), lmax = -__builtin_inf();
  for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < n; i += (int64_t)gridDim.x * 4) {
    double off = 0.0, dg = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
      const double v = (double)bf16_val(hi[i * ld + j]) + (double)bf16_val(lo[i * ld + j]);
      if (j == i) dg = v; else off += fabs(v);
    }
    off = wave_sum(off);
    dg = wave_sum(dg);
    lmin = fmin(lmin, dg - off);
    lmax = fmax(lmax, dg + off);
  }
  if (lane == 0) {
    sl[wave] = lmin;
    sh[wave] = lmax;
  }
  __syncthreads();
  if (tid == 0) {
    part[2 * blockIdx.x] = fmin(fmin(sl[0], sl[1]), fmin(sl[2], sl[3]));
    part[2 * blockIdx.x + 1] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  }
}

static __global__ __launch_bounds__(64) void k_gersh_finish(Ctl* __restrict__ ctl, const double* __restrict__ part,
                                                     int nwg) {
  double lmin = __builtin_inf(), lmax = -__builtin_inf();
  for (int w = threadIdx.x; w < nwg; w += 64) {
    lmin = fmin(lmin, part[2 * w]);
    lmax = fmax(lmax, part[2 * w + 1]);
  }
  lmin = wave_min(lmin);
  lmax = wave_max(lmax);
  if (threadIdx.x == 0) {
    ctl->op_lmin = lmin;
    ctl->op_lmax = lmax;
  }
}

// What the server reads back after a launch, per slot.
struct SlotSummary {
  int64_t t;
  int32_t stop, status;
  int32_t barerr, reserved;  // the team's barrier error flag
  Info info;
};

template <typename T>
static __global__ __launch_bounds__(256) void k_serve_summary(const Slot<T>* __restrict__ slots, int nslots,
                                                       SlotSummary* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nslots) return;
  const Ctl* c = slots[i].ctl;
  if (!c) return;
  SlotSummary s;
  s.t = c->t;
  s.stop = c->stop;
  s.status = c->status;
  s.barerr = (int32_t)slots[i].b.bar[kBarErr];
  s.reserved = 0;
  s.info = c->info;
  out[i] = s;
}

// ---------------------------------------------------------------------------
// caller-supplied gradient: Gershgorin bounds of G_t (per workgroup min of
// g_ii - sum_{j != i} |g_ij| and max of g_ii + sum_{j != i} |g_ij|, FP64
// sums, one wave per row) -> part[2 wg], part[2 wg + 1]; then the step
// scalars of the step with those bounds
// ---------------------------------------------------------------------------
template <typename T>
static __global__ __launch_bounds__(256) void k_gersh_dense(const T* __restrict__ D, int64_t n, int64_t ld,
                                                            double* __restrict__ part) {
  __shared__ double sl[4], sh[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double lmin = __builtin_inf(), lmax = -__builtin_inf();
  for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < n; i += (int64_t)gridDim.x * 4) {
    double off = 0.0, dg = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
      const double v = (double)D[i * ld + j];
      if (j == i) dg = v; else off += fabs(v);
    }
    off = wave_sum(off);
    dg = wave_sum(dg);
    lmin = fmin(lmin, dg - off);
    lmax = fmax(lmax, dg + off);
  }
  if (lane == 0) {
    sl[wave] = lmin;
    sh[wave] = lmax;
  }
  __syncthreads();
  if (tid == 0) {
    part[2 * blockIdx.x] = fmin(fmin(sl[0], sl[1]), fmin(sl[2], sl[3]));
    part[2 * blockIdx.x + 1] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  }
}

template <typename T>
static __global__ __launch_bounds__(256) void k_gersh_csr(const int* __restrict__ rp, const int* __restrict__ col,
                                                          const T* __restrict__ val, int64_t n,
                                                          double* __restrict__ part) {
  __shared__ double sl[4], sh[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double lmin = __builtin_inf(), lmax = -__builtin_inf();
  for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < n; i += (int64_t)gridDim.x * 4) {
    double off = 0.0, dg = 0.0;
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) {
      const double v = (double)val[e];
      if (col[e] == i) dg += v; else off += fabs(v);
    }
    off = wave_sum(off);
    dg = wave_sum(dg);
    lmin = fmin(lmin, dg - off);
    lmax = fmax(lmax, dg + off);
  }
  if (lane == 0) {
    sl[wave] = lmin;
    sh[wave] = lmax;
  }
  __syncthreads();
  if (tid == 0) {
    part[2 * blockIdx.x] = fmin(fmin(sl[0], sl[1]), fmin(sl[2], sl[3]));
    part[2 * blockIdx.x + 1] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  }
}

// op_lmin/op_lmax of this step's G_t from the partial bounds, then the step
// scalars (shift and coefficients) for it; one wavefront
static __global__ __launch_bounds__(64) void k_external_setup(Cfg cfg, Ctl* __restrict__ ctl,
                                                              const double* __restrict__ part, int nwg) {
  const int lane = threadIdx.x;
  double lmin = __builtin_inf(), lmax = -__builtin_inf();
  for (int w = lane; w < nwg; w += 64) {
    lmin = fmin(lmin, part[2 * w]);
    lmax = fmax(lmax, part[2 * w + 1]);
  }
  lmin = wave_min(lmin);
  lmax = wave_max(lmax);
  if (lane == 0) {
    ctl->op_lmin = lmin;
    ctl->op_lmax = lmax;
  }
  wg_fence();
  step_scalars(cfg, (gbl<Ctl>*)ctl, lane);
}

// minibatch indices in [0, m)
static __global__ __launch_bounds__(256) void k_check_idx(const int* __restrict__ idx, int64_t cnt, int64_t m,
                                                   int* __restrict__ err) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    const int v = idx[e];
    if (v < 0 || (int64_t)v >= m) *err = 1;
  }
}

static __global__ __launch_bounds__(256) void k_check_csr(const int* __restrict__ rp, const int* __restrict__ col,
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
