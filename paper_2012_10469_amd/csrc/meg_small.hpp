// Small k x k FP64 solves of the subspace iteration, run by ONE wavefront
// (lanes 0..63 of the workgroup that completes a grid barrier):
//   Rayleigh-Ritz on the current subspace (Section 3: eigenpairs of W^T M W),
//   the Cholesky-QR transform that orthonormalises the next block, and, at the
//   end of the inner solve, the exponentiation / normalisation of Definition 1
//   and the cheap certificate with b_{r+1} (Section 3.1.1).
// The wavefront works wave-synchronously: no workgroup barriers, only
// wavefront-scope fences between dependent LDS phases.  Matrices live in LDS
// with row stride KB + 1.
#pragma once
#include "meg_device.hpp"

namespace meg {

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// C = op(A) B for KB x KB matrices in LDS (stride KB + 1), op(A) = A or A^T,
// on the FP64 matrix cores: 16 x 16 output tiles, v_mfma_f64_16x16x4f64 per
// 4-wide K step.  Lane layout: A operand lane l holds A[l % 16][l / 16], B
// operand lane l holds B[l / 16][l % 16], result register v of lane l is
// C[l / 16 + 4 v][l % 16].  All 64 lanes must call it.  C may not alias A
// or B (results are written after all reads of a tile).
typedef double f64x4_t __attribute__((ext_vector_type(4)));
template <int KB, bool TA>
__device__ __forceinline__ void mm_mfma(const lds<double>* A, const lds<double>* B, lds<double>* C, int lane) {
  constexpr int LD = KB + 1;
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < KB / 16; ++ti)
#pragma unroll
    for (int tj = 0; tj < KB / 16; ++tj) {
      f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KB / 4; ++s) {
        const int k = 4 * s + kq;
        const double a = TA ? A[k * LD + 16 * ti + i] : A[(16 * ti + i) * LD + k];
        const double b = B[k * LD + 16 * tj + i];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) C[(16 * ti + kq + 4 * v) * LD + 16 * tj + i] = acc[v];
    }
}

// C = A^T B (all KB x KB, LDS stride KB + 1)
template <int KB>
__device__ __forceinline__ void mm_tn(const lds<double>* A, const lds<double>* B, lds<double>* C, int lane) {
  mm_mfma<KB, true>(A, B, C, lane);
}

// C = A B
template <int KB>
__device__ __forceinline__ void mm_nn(const lds<double>* A, const lds<double>* B, lds<double>* C, int lane) {
  mm_mfma<KB, false>(A, B, C, lane);
}

// dense KB x KB (stride KB, global) <-> LDS stride KB + 1; the loops have
// compile-time trip counts so all loads are issued before any is used
template <int KB>
__device__ __forceinline__ void load_mat(const gbl<double>* src, lds<double>* dst, int lane) {
  constexpr int IT = KB * KB / 64;
  double v[IT];
#pragma unroll
  for (int u = 0; u < IT; ++u) v[u] = src[lane + 64 * u];
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int e = lane + 64 * u;
    dst[(e / KB) * (KB + 1) + (e % KB)] = v[u];
  }
}

// symmetric KB x KB from its upper triangle by rows (PartRec) -> LDS
// stride KB + 1, both triangles; all loads issued before any is stored
template <int KB>
__device__ __forceinline__ void load_sym(const gbl<double>* src, lds<double>* dst, int lane) {
  constexpr int IT = KB * KB / 64;
  double v[IT];
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int e = lane + 64 * u, i = e / KB, j = e % KB;
    v[u] = src[i <= j ? PartRec<KB>::tri(i, j) : PartRec<KB>::tri(j, i)];
  }
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int e = lane + 64 * u;
    dst[(e / KB) * (KB + 1) + (e % KB)] = v[u];
  }
}

template <int KB>
__device__ __forceinline__ void store_mat(const lds<double>* src, gbl<double>* dst, int lane) {
#pragma unroll
  for (int u = 0; u < KB * KB / 64; ++u) {
    const int e = lane + 64 * u;
    dst[e] = src[(e / KB) * (KB + 1) + (e % KB)];
  }
}

// dst[e] = src[e], e < KB * KB (global to global), all loads in flight
template <int KB>
__device__ __forceinline__ void copy_mat(const gbl<double>* src, gbl<double>* dst, int lane) {
  constexpr int IT = KB * KB / 64;
  double v[IT];
#pragma unroll
  for (int u = 0; u < IT; ++u) v[u] = src[lane + 64 * u];
#pragma unroll
  for (int u = 0; u < IT; ++u) dst[lane + 64 * u] = v[u];
}

// 1/sqrt(x) and 1/x in FP64 from the hardware estimates plus one Newton step
// (relative error ~1e-16 for normal x > 0).
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * (1.5 - 0.5 * x * y * y);
}
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return y * (2.0 - x * y);
}

// Value of v in lane l (0 <= l < 16, a compile-time constant once unrolled)
// of this lane's row of 16 lanes: one 64-bit DPP move (row_newbcast).
__device__ __forceinline__ double row_bcast_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  long long x = b;
  switch (l) {
#define MEG_ROW_BCAST(n) \
  case n: x = __builtin_amdgcn_mov_dpp(b, 0x150 + n, 0xF, 0xF, false); break;
    MEG_ROW_BCAST(0) MEG_ROW_BCAST(1) MEG_ROW_BCAST(2) MEG_ROW_BCAST(3) MEG_ROW_BCAST(4) MEG_ROW_BCAST(5)
    MEG_ROW_BCAST(6) MEG_ROW_BCAST(7) MEG_ROW_BCAST(8) MEG_ROW_BCAST(9) MEG_ROW_BCAST(10) MEG_ROW_BCAST(11)
    MEG_ROW_BCAST(12) MEG_ROW_BCAST(13) MEG_ROW_BCAST(14) MEG_ROW_BCAST(15)
#undef MEG_ROW_BCAST
  }
  return __longlong_as_double(x);
}

// Jacobi rotation zeroing A_pq of the 2 x 2 block [[app, apq], [apq, aqq]]:
//   t = tan(angle) = 2 apq sign(delta) / (|delta| + sqrt(delta^2 + 4 apq^2)),
//   delta = aqq - app, c = 1/sqrt(1 + t^2), s = t c
// (the smaller of the two angles; no division by apq, so no overflow case).
// Branch-free, so the rotations a lane needs interleave.  Identity when A_pq
// is negligible.
__device__ __forceinline__ void jacobi_rot(double app, double aqq, double apq, double& c, double& s) {
  const bool act = apq * apq > 1e-36 * fabs(app * aqq) && fabs(apq) > 1e-300;
  const double b = act ? apq : 0.0;
  const double delta = aqq - app;
  const double r2 = fmax(delta * delta + 4.0 * b * b, 1e-300);
  const double r = r2 * rsqrt_nr(r2);
  const double den = fmax(fabs(delta) + r, 1e-300);
  const double t = 2.0 * (delta >= 0.0 ? b : -b) * rcp_nr(den);
  c = rsqrt_nr(1.0 + t * t);
  s = t * c;
}

// The same rotation with its angle from FP32 arithmetic (hardware square
// root and reciprocal, no refinement): t carries a relative error of ~1e-7,
// which leaves |A_pq| ~ 1e-7 |A_pq| after the rotation (the next sweep
// removes it; an FP32 state's tolerance is 1e-8 relative), while c and s
// are formed from that t in FP64, so c^2 + s^2 = 1 to FP64 rounding and S
// stays orthogonal to FP64 accuracy.  The pair's entries are far inside the
// FP32 range here (eigenvalues of the shifted step operator).
__device__ __forceinline__ void jacobi_rot_f32angle(double app, double aqq, double apq, double& c, double& s) {
  const bool act = apq * apq > 1e-36 * fabs(app * aqq) && fabs(apq) > 1e-300;
  const float bf = act ? (float)apq : 0.0f;
  const float df = (float)(aqq - app);
  const float rf = __builtin_amdgcn_sqrtf(fmaf(df, df, 4.0f * bf * bf));
  const float den = fmaxf(fabsf(df) + rf, 1e-37f);
  const double t = (double)(2.0f * (df >= 0.0f ? bf : -bf) * __builtin_amdgcn_rcpf(den));
  c = rsqrt_nr(1.0 + t * t);
  s = t * c;
}
template <bool F32ANGLE>
__device__ __forceinline__ void jacobi_rot_sel(double app, double aqq, double apq, double& c, double& s) {
  if constexpr (F32ANGLE) jacobi_rot_f32angle(app, aqq, apq, c, s); else jacobi_rot(app, aqq, apq, c, s);
}

// Circle-method ordering: slot j sits at position j in round 0; slot 0 stays
// at 0, the others move up by one position per round, wrapping from KB - 1 to
// 1.  Rotation m pairs the positions of slots m and KB - 1 - m.
template <int KB>
__device__ __forceinline__ int jacobi_next(int pos) { return pos == 0 ? 0 : (pos == KB - 1 ? 1 : pos + 1); }

// Cyclic parallel Jacobi as below, for blocks larger than 16: the KB/2
// rotations of a round are computed once (lane m < KB/2 computes rotation m)
// into LDS (`rot`, 2 * KB doubles: c, s, then the pair's positions), then
// every lane updates its 2 x 2 blocks.  Lane l owns the blocks (m1, m2) with
// m2 = l % (KB/2) and m1 = l / (KB/2) + (64 / (KB/2)) b, so it reads rotation
// m2 once per round.  Blocks are disjoint, so all of a lane's reads precede
// its writes.
template <int KB, bool F32ANGLE>
__device__ __noinline__ int jacobi_shared_rot(lds<double>* A, lds<double>* S, double off2_tol, int lane,
                                              lds<double>* rot) {
  constexpr int LD = KB + 1;
  constexpr int NP = KB / 2;
  constexpr int BPL = NP * NP / 64;
  static_assert(64 % NP == 0, "whole rows of blocks per lane group");
  for (int e = lane; e < KB * KB; e += 64) S[(e / KB) * LD + (e % KB)] = (e / KB == e % KB) ? 1.0 : 0.0;
  wsync();
  const int m2 = lane % NP;
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < KB * KB; e += 64) {
      const double v = A[(e / KB) * LD + (e % KB)];
      if (e / KB == e % KB) dia += v * v; else off += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if (!(off > off2_tol * (off + dia))) break;  // also exits on NaN
    int am = lane, bm = KB - 1 - lane;  // positions of slots m and KB - 1 - m (lanes m < NP)
    for (int round = 0; round < KB - 1; ++round) {
      if (lane < NP) {
        const int p = min(am, bm), q = max(am, bm);
        double c, s;
        jacobi_rot_sel<F32ANGLE>(A[p * LD + p], A[q * LD + q], A[p * LD + q], c, s);
        rot[2 * lane] = c;
        rot[2 * lane + 1] = s;
        rot[KB + 2 * lane] = p;  // indices kept beside the rotation (exact in FP64)
        rot[KB + 2 * lane + 1] = q;
      }
      am = jacobi_next<KB>(am);
      bm = jacobi_next<KB>(bm);
      wsync();
      const double c2 = rot[2 * m2], s2 = rot[2 * m2 + 1];
      const int p2 = (int)rot[KB + 2 * m2], q2 = (int)rot[KB + 2 * m2 + 1];
      double c1[BPL], s1[BPL], a[BPL], b[BPL], cc[BPL], d[BPL], sx[BPL][2], sy[BPL][2];
      int p1[BPL], q1[BPL];
#pragma unroll
      for (int bi = 0; bi < BPL; ++bi) {
        const int m1 = lane / NP + (64 / NP) * bi;
        c1[bi] = rot[2 * m1];
        s1[bi] = rot[2 * m1 + 1];
        p1[bi] = (int)rot[KB + 2 * m1];
        q1[bi] = (int)rot[KB + 2 * m1 + 1];
      }
#pragma unroll
      for (int bi = 0; bi < BPL; ++bi) {
        a[bi] = A[p1[bi] * LD + p2];
        b[bi] = A[p1[bi] * LD + q2];
        cc[bi] = A[q1[bi] * LD + p2];
        d[bi] = A[q1[bi] * LD + q2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // S <- S J1 in rows 2 m2, 2 m2 + 1
          const int row = 2 * m2 + h;
          sx[bi][h] = S[row * LD + p1[bi]];
          sy[bi][h] = S[row * LD + q1[bi]];
        }
      }
#pragma unroll
      for (int bi = 0; bi < BPL; ++bi) {
        const double ra = c1[bi] * a[bi] - s1[bi] * cc[bi], rb = c1[bi] * b[bi] - s1[bi] * d[bi];  // rows: J1^T
        const double rc = s1[bi] * a[bi] + c1[bi] * cc[bi], rd = s1[bi] * b[bi] + c1[bi] * d[bi];
        A[p1[bi] * LD + p2] = c2 * ra - s2 * rb;                                                // columns: J2
        A[p1[bi] * LD + q2] = s2 * ra + c2 * rb;
        A[q1[bi] * LD + p2] = c2 * rc - s2 * rd;
        A[q1[bi] * LD + q2] = s2 * rc + c2 * rd;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int row = 2 * m2 + h;
          S[row * LD + p1[bi]] = c1[bi] * sx[bi][h] - s1[bi] * sy[bi][h];
          S[row * LD + q1[bi]] = s1[bi] * sx[bi][h] + c1[bi] * sy[bi][h];
        }
      }
      wsync();
    }
  }
  return sweep;
}

// Storage slot of circle position x: the pair of positions m and KB - 1 - m
// (rotation m of every round) is kept in slots 2m and 2m + 1.
// jacobi_slot_move(s): the slot that the entry in slot s moves to for the
// next round, the slot of the position before its own (the inverse of
// jacobi_next), so that round t pairs the indices next^t(m) and
// next^t(KB - 1 - m), the pairs of the ordering above.  A full sweep of
// KB - 1 rounds moves every entry once around its cycle, back to its slot.
template <int KB>
__device__ __forceinline__ int jacobi_slot(int x) { return x < KB / 2 ? 2 * x : 2 * (KB - 1 - x) + 1; }
template <int KB>
__device__ __forceinline__ int jacobi_slot_move(int s) {
  const int m = s >> 1;
  const int x = (s & 1) ? KB - 1 - m : m;
  return jacobi_slot<KB>(x == 0 ? 0 : (x == 1 ? KB - 1 : x - 1));
}

// Cyclic parallel Jacobi (round-robin ordering) for symmetric A in LDS.
// On return A is (numerically) diagonal and A_in = S diag(A) S^T.  Stops
// when the off-diagonal mass is below off2_tol of the total (squared norms);
// returns the number of sweeps taken.  Each round applies KB/2 disjoint
// rotations J_m, rotation m on the indices held in slots 2m and 2m + 1.  A
// lane owns the 2 x 2 block (m1, m2) of A, updated as J_m1^T A_{m1 m2} J_m2,
// and the S entries of rotation m1 in rows 2 m2 and 2 m2 + 1.  It computes
// its column rotation m2 itself from that pair's diagonal block (the same
// inputs and operations in every lane, so every lane derives the same
// rotation); its row rotation m1 is the column rotation of lane 8 m1, which
// owns the block (m1, m1) (lane = 8 m1 + (m2 - m1) mod 8 puts it at position
// 0 or 8 of the row of 16 lanes that holds all of pair m1's blocks), and
// arrives by two fixed row broadcasts.  Index x starts in
// slot jacobi_slot(x) (A permuted on entry, S the matching permutation, so
// A_in = S A S^T throughout), and the rotated entries are stored where the
// next round's pairing wants them (rows and columns of A, columns of S moved
// by jacobi_slot_move): every lane reads and writes the same LDS locations
// in every round.  All loads of a round precede its stores (in-order LDS
// queue of the wavefront).
template <int KB, bool F32ANGLE>
__device__ __noinline__ int jacobi(lds<double>* A, lds<double>* S, double off2_tol, int lane, lds<double>* rot) {
  constexpr int LD = KB + 1;
  constexpr int NP = KB / 2;
  static_assert((NP * NP) % 64 == 0, "2 x 2 blocks must fill the wavefront");
  constexpr int BPL = NP * NP / 64;  // 2 x 2 blocks per lane
  if constexpr (BPL > 1) {
    return jacobi_shared_rot<KB, F32ANGLE>(A, S, off2_tol, lane, rot);
  } else {
    constexpr int IT = KB * KB / 64;
    double v[IT];
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int e = lane + 64 * u;
      v[u] = A[(e / KB) * LD + (e % KB)];
    }
    __asm__ volatile("" ::: "memory");  // every entry read before any is moved
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int e = lane + 64 * u, i = e / KB, j = e % KB;
      A[jacobi_slot<KB>(i) * LD + jacobi_slot<KB>(j)] = v[u];
      S[i * LD + j] = (j == jacobi_slot<KB>(i)) ? 1.0 : 0.0;
    }
    const unsigned m1 = (unsigned)lane / NP, m2 = ((unsigned)lane % NP + m1) % NP;
    const bool odd = (m1 & 1u) != 0;  // lane 8 m1 sits at position 8 of its row
    // read locations (fixed): the block, the column pair's diagonal block, S
    const unsigned rb = (2 * m1) * LD + 2 * m2;
    const unsigned d2 = (2 * m2) * (LD + 1);
    const unsigned sr = (2 * m2) * LD + 2 * m1;
    // write locations: the block's rows and columns, S's columns, moved on
    const unsigned r0 = jacobi_slot_move<KB>(2 * m1), r1 = jacobi_slot_move<KB>(2 * m1 + 1);
    const unsigned c0 = jacobi_slot_move<KB>(2 * m2), c1 = jacobi_slot_move<KB>(2 * m2 + 1);
    const unsigned w00 = r0 * LD + c0, w01 = r0 * LD + c1, w10 = r1 * LD + c0, w11 = r1 * LD + c1;
    const unsigned s0 = (2 * m2) * LD + r0, s1 = (2 * m2) * LD + r1;
    wsync();
    int sweep = 0;
    for (; sweep < 30; ++sweep) {
      double off = 0.0, dia = 0.0;
      for (int e = lane; e < KB * KB; e += 64) {
        const double v = A[(e / KB) * LD + (e % KB)];
        if (e / KB == e % KB) dia += v * v; else off += v * v;
      }
      off = wave_sum(off);
      dia = wave_sum(dia);
      if (!(off > off2_tol * (off + dia))) break;  // also exits on NaN
      for (int round = 0; round < KB - 1; ++round) {
        const double a = A[rb], b = A[rb + 1], cc = A[rb + LD], d = A[rb + LD + 1];
        const double p2 = A[d2], q2 = A[d2 + LD + 1], o2 = A[d2 + 1];
        const double sx0 = S[sr], sy0 = S[sr + 1], sx1 = S[sr + LD], sy1 = S[sr + LD + 1];
        __asm__ volatile("" ::: "memory");  // this round's loads, then its stores
        double cs2, sn2;
        jacobi_rot_sel<F32ANGLE>(p2, q2, o2, cs2, sn2);
        const double ce = row_bcast_f64(cs2, 0), co = row_bcast_f64(cs2, 8);
        const double se = row_bcast_f64(sn2, 0), so = row_bcast_f64(sn2, 8);
        const double cs1 = odd ? co : ce, sn1 = odd ? so : se;
        const double ra = cs1 * a - sn1 * cc, rbv = cs1 * b - sn1 * d;  // rows: J1^T
        const double rc = sn1 * a + cs1 * cc, rd = sn1 * b + cs1 * d;
        A[w00] = cs2 * ra - sn2 * rbv;                                  // columns: J2
        A[w01] = sn2 * ra + cs2 * rbv;
        A[w10] = cs2 * rc - sn2 * rd;
        A[w11] = sn2 * rc + cs2 * rd;
        S[s0] = cs1 * sx0 - sn1 * sy0;  // S <- S J1 in rows 2 m2, 2 m2 + 1
        S[s1] = sn1 * sx0 + cs1 * sy0;
        S[s0 + LD] = cs1 * sx1 - sn1 * sy1;
        S[s1 + LD] = sn1 * sx1 + cs1 * sy1;
        wsync();
      }
    }
    return sweep;
  }
}

// Value of v in lane l (l uniform across the wavefront), as a scalar.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky A = R^T R (R upper) of the symmetric positive definite A (LDS,
// upper triangle read), R written to LDS (stride KB + 1, zero below the
// diagonal) and the reciprocals of its diagonal to rdiag[0, KB).  Lane c
// holds column c in registers; every value another lane needs is a readlane
// of a compile-time lane index, so the factorisation touches no memory until
// R is stored.  Tiny pivots are floored to keep R invertible.
template <int KB>
__device__ __noinline__ void chol_factor(const lds<double>* A, lds<double>* R, lds<double>* rdiag, int lane) {
  constexpr int LD = KB + 1;
  const int col = lane < KB ? lane : KB - 1;
  // column `lane` of A, overwritten by column `lane` of R; its entries below
  // the diagonal (i > lane) are loaded too (one batch of loads, no select
  // the compiler could turn into a branch per load) but never read, and
  // lanes past KB hold a copy of the last column
  double a[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i) a[i] = A[i * LD + col];
  const double scale = wave_max(lane < KB ? A[col * LD + col] : 0.0);
  const double floor_piv = fmax(scale, 1e-300) * 1e-28;
  if constexpr (KB == 16) {
    // The 16 columns are the lanes of one DPP row: row j of the trailing
    // matrix reaches every lane by 64-bit row broadcasts, taken before row j
    // is scaled, so they do not wait for the pivot's square root.  Step j
    // subtracts A_ji A_jc / d_j (d_j the pivot) from A_ic, then scales row j
    // into R (R_jc = A_jc / sqrt(d_j), R_jj = sqrt(d_j)).
    double rd = 0.0;  // 1 / R_cc in lane c
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      double bj[KB];
#pragma unroll
      for (int i = j; i < KB; ++i) bj[i] = row_bcast_f64(a[j], i);
      double dj = bj[j];
      if (!(dj > floor_piv)) dj = floor_piv;
      const double rinv = rsqrt_nr(dj);
      const double f = a[j] * (rinv * rinv);
#pragma unroll
      for (int i = j + 1; i < KB; ++i) {
        // A_ic -= A_ji A_jc / d_j (A_ji held by lane i).  Done in every lane:
        // the entries below a lane's diagonal (i > c) are never read.
        a[i] -= bj[i] * f;
      }
      a[j] = (lane == j) ? dj * rinv : a[j] * rinv;
      rd = (lane == j) ? rinv : rd;
    }
    if (lane < KB) {
#pragma unroll
      for (int i = 0; i < KB; ++i) R[i * LD + lane] = (i <= lane) ? a[i] : 0.0;
      rdiag[lane] = rd;
    }
  } else {
    double rd = 0.0;  // 1 / R_cc in lane c
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      double dj = readlane_d(a[j], j);
      if (!(dj > floor_piv)) dj = floor_piv;
      const double rinv = rsqrt_nr(dj);
      // row j of R: R_jj = sqrt(dj) (lane j), R_jc = A_jc / R_jj (lanes c > j)
      a[j] = (lane == j) ? dj * rinv : a[j] * rinv;
      rd = (lane == j) ? rinv : rd;
#pragma unroll
      for (int i = j + 1; i < KB; ++i) {
        // A_ic -= R_ji R_jc (R_ji held by lane i).  Done in every lane: the
        // entries below a lane's diagonal (i > c) are never read.
        a[i] -= readlane_d(a[j], i) * a[j];
      }
    }
    if (lane < KB) {
#pragma unroll
      for (int i = 0; i < KB; ++i) R[i * LD + lane] = (i <= lane) ? a[i] : 0.0;
      rdiag[lane] = rd;
    }
  }
  wsync();
}

// Y = X R^{-1} for the first `rows` (<= 64) rows of X (LDS, stride KB + 1; Y
// may be X) with R upper triangular (LDS, as chol_factor leaves it): lane i
// solves y R = x_i by forward substitution, y_j = (x_ij - sum_{m<j} y_m R_mj)
// / R_jj, subtracting each y_j from the later columns as soon as it is known.
// Every lane reads the same entries of R at the same time (LDS broadcasts).
template <int KB>
__device__ __noinline__ void rsolve(const lds<double>* X, lds<double>* Y, const lds<double>* R,
                                    const lds<double>* rdiag, int rows, int lane) {
  constexpr int LD = KB + 1;
  const bool act = lane < rows;
  const int row = act ? lane : rows - 1;  // lanes past the rows solve a copy of the last one
  double y[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) y[j] = X[row * LD + j];
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    // R is consumed two rows at a time: the running values are pinned and
    // memory is fenced for the compiler here, so later rows are not read
    // ahead into registers (all of R would not fit)
    if (j % 2 == 0) {
#pragma unroll
      for (int i = 0; i < KB; ++i) __asm__ volatile("" : "+v"(y[i])::"memory");
    }
    y[j] *= rdiag[j];
#pragma unroll
    for (int i = j + 1; i < KB; ++i) y[i] -= y[j] * R[j * LD + i];
  }
  wsync();  // every lane has read its row before any row is written (Y may be X)
  if (act) {
#pragma unroll
    for (int j = 0; j < KB; ++j) Y[lane * LD + j] = y[j];
  }
  wsync();
}

// The 16 x 16 case of chol_apply2 in one pass over the factorisation: every
// row of 16 lanes factors A = R^T R (lane c of the row holding column c, as
// chol_factor does) and lane l < 32 carries row l of [X1; X2] through the
// forward substitution y R = x alongside it.  Step j's row broadcasts of the
// trailing matrix (A_ji, lane i) serve both: R_ji = A_ji / sqrt(d_j), so
// y_i -= y_j R_ji needs no further exchange.  R itself is not stored.
__device__ __noinline__ void chol_solve16(const lds<double>* A, lds<double>* X1, int lane) {
  constexpr int KB = 16, LD = KB + 1;
  const int col = lane & (KB - 1);
  const int row = lane < 2 * KB ? lane : 2 * KB - 1;  // lanes past the rows solve a copy of the last one
  double a[KB], y[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    a[i] = A[i * LD + col];  // entries below the diagonal (i > col) are never read
    y[i] = X1[row * LD + i];
  }
  const double scale = wave_max(A[col * LD + col]);
  const double floor_piv = fmax(scale, 1e-300) * 1e-28;
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    double bj[KB];
#pragma unroll
    for (int i = j; i < KB; ++i) bj[i] = row_bcast_f64(a[j], i);
    double dj = bj[j];
    if (!(dj > floor_piv)) dj = floor_piv;
    const double rinv = rsqrt_nr(dj);
    const double f = a[j] * (rinv * rinv);  // A_jc / d_j
    const double yj = y[j] * rinv;          // y_j = (x_j - sum_{m<j} y_m R_mj) / R_jj
    const double g = yj * rinv;
    y[j] = yj;
#pragma unroll
    for (int i = j + 1; i < KB; ++i) {
      a[i] -= bj[i] * f;  // trailing update (entries below a lane's diagonal unused)
      y[i] -= bj[i] * g;  // y_j R_ji
    }
    // both recurrences advance together, one step at a time: otherwise the
    // compiler runs the factorisation ahead of the substitution and holds
    // every step's broadcasts in registers
#pragma unroll
    for (int i = j; i < KB; ++i) __asm__ volatile("" : "+v"(a[i]), "+v"(y[i]));
  }
  wsync();  // every lane has read its row (and A) before any row is written
  if (lane < 2 * KB) {
#pragma unroll
    for (int i = 0; i < KB; ++i) X1[lane * LD + i] = y[i];
  }
  wsync();
}

// Rows [X1; X2] (2 KB rows from X1, X2 = X1 + KB * (KB + 1)) times R^{-1}
// in place, for R the Cholesky factor of the Gram matrix A: the
// orthonormalising transform applied to two KB x KB blocks at once.  Rscr:
// KB * (KB + 1) doubles for R, rdiag: KB doubles (scratch; not written for
// KB = 16).
template <int KB>
__device__ __forceinline__ void chol_apply2(const lds<double>* A, lds<double>* X1, lds<double>* Rscr,
                                            lds<double>* rdiag, int lane) {
  if constexpr (KB == 16) {
    chol_solve16(A, X1, lane);
  } else {
    chol_factor<KB>(A, Rscr, rdiag, lane);
    if constexpr (2 * KB <= 64) {
      rsolve<KB>(X1, X1, Rscr, rdiag, 2 * KB, lane);
    } else {
      rsolve<KB>(X1, X1, Rscr, rdiag, KB, lane);
      rsolve<KB>(X1 + KB * (KB + 1), X1 + KB * (KB + 1), Rscr, rdiag, KB, lane);
    }
  }
}

// Per-step operator coefficients: Yhat = V diag(ceff) V^T + opscale*Op + sdiag*I
// equals M_t - log(alpha) I + sigma I.  gmax is an upper bound of
// lambda_max(grad f(X_t)); by Weyl's inequality
//   lambda_min(V diag(c) V^T - eta G) >= min(0, min c) - eta gmax,
// so sigma = eta gmax - min(0, min c) (+ a small margin) makes Yhat >= 0 and
// subspace iteration targets the algebraically largest eigenvalues.  A tight
// gmax matters: the unwanted spectrum then starts near 0, which is what makes
// the (r+1)-th pair converge.  One wavefront (all 64 lanes call it).
// setup_step_v takes the iterate's alpha, d_l and c_l (lane l < r; zero
// elsewhere) from the caller, setup_step reads them from ctl.
// mu_1, mu_k: the last step's extreme Ritz values as eigenvalues of M
// (mu_valid 0: none), for the first sweep's Chebyshev interval.
__device__ inline void setup_step_v(const Cfg& cfg, gbl<Ctl>* ctl, double gmax, double alpha, double dl, double cl,
                                    double mu_1, double mu_k, int mu_valid, int lane) {
  const int r = cfg.r;
  const bool act = lane < r;
  const double cmin = wave_min(act ? fmin(cl, 0.0) : 0.0);
  const double cmax = wave_max(act ? fmax(cl, 0.0) : 0.0);
  const double base = cfg.eta * gmax - cmin;
  const double sigma = base + 1e-3 * (fabs(base) + cmax) + 1e-30;
  const bool den = cfg.kind == DENOISE_DENSE;
  if (lane < KMAX) {
    // denoising, G = X - M:  V c V^T - eta(alpha I + V d V^T - M) + sigma I
    ctl->ceff[lane] = act ? (den ? cl - cfg.eta * dl : cl) : 0.0;
  }
  if (lane == 0) {
    ctl->gmax = gmax;
    ctl->sigma = sigma;
    ctl->sdiag = den ? sigma - cfg.eta * alpha : sigma;
    ctl->opscale = den ? cfg.eta : -cfg.eta;
    // the first sweep's Chebyshev interval [0, b]: the last step's mu_k,
    // shifted as this step's operator is (Yhat = M_t - log alpha + sigma)
    double b = 0.0;
    if (cfg.cheb && mu_valid) {
      const double la = log(alpha);
      const double bk = mu_k - la + sigma, b1 = mu_1 - la + sigma;
      if (bk > 1e-3 * b1 && bk < 0.5 * b1) b = bk;
    }
    ctl->cheb_b = b;
  }
}
__device__ inline void setup_step(const Cfg& cfg, gbl<Ctl>* ctl, double gmax, int lane) {
  const bool act = lane < cfg.r;
  setup_step_v(cfg, ctl, gmax, ctl->alpha, act ? ctl->d[lane] : 0.0, act ? ctl->c[lane] : 0.0, ctl->mu_1, ctl->mu_k,
               ctl->mu_valid, lane);
}

// gmax >= lambda_max(grad f(X_t)) for the objectives whose bound needs no pass
// over the data (the bounds are derived at step_scalars); dl = d_l (lane
// l < r, zero elsewhere).  One wavefront.
__device__ inline double grad_bound(const Cfg& cfg, double alpha, double dl, double op_lmin, double op_lmax,
                                    int pxvalid, double pxnorm, double dxnorm, int lane) {
  const bool act = lane < cfg.r;
  if (cfg.kind == DENOISE_DENSE) return alpha + wave_max(act ? fmax(dl, 0.0) : 0.0) - op_lmin;
  if (cfg.kind == MASKED_CSR) {
    const double ev = alpha + dl;
    const double fro2 = (double)(cfg.n - cfg.r) * alpha * alpha + wave_sum(act ? ev * ev : 0.0);
    const double px = pxvalid ? fmin(pxnorm + dxnorm, sqrt(fro2)) : sqrt(fro2);
    return px - op_lmin;
  }
  return op_lmax;
}

// The step's scalars that the small solve reads, loaded once at its start
// (together with its matrices) instead of at their points of use, where
// each read would be a separate round trip to memory.
struct SolveScalars {
  double alpha, sigma, solve_tol, f, pxnorm, op_lmin, op_lmax, dl;  // dl: d_l of this lane (l < r)
  double mu_up_raw;  // an upper bound of mu_{r+1} armed for step mu_up_t (see up_bound)
  double cheb_b, xscale;
  int64_t t, iters, applies, jacobi, extrap_n, unconv_n, mu_up_t;
  int fvalid, pxvalid, polish, xvalid;
  // the bound of mu_{r+1} for this step (+inf: none armed for it); decided at
  // the point of use, so that loading the scalars waits for none of them
  __device__ double up_bound() const { return (mu_up_t == t && t > 0) ? mu_up_raw : __builtin_inf(); }
};
__device__ __forceinline__ SolveScalars load_scalars(const Cfg& cfg, const gbl<Ctl>* ctl, int lane) {
  SolveScalars s;
  s.alpha = ctl->alpha;
  s.sigma = ctl->sigma;
  s.solve_tol = ctl->solve_tol;
  s.f = ctl->f;
  s.pxnorm = ctl->pxnorm;
  s.op_lmin = ctl->op_lmin;
  s.op_lmax = ctl->op_lmax;
  s.dl = (lane < cfg.r) ? ctl->d[lane] : 0.0;
  s.t = ctl->t;
  s.mu_up_raw = ctl->mu_up;  // read unconditionally: one round trip with the rest
  s.mu_up_t = ctl->mu_up_t;
  s.cheb_b = ctl->cheb_b;
  s.xscale = ctl->xscale;
  s.iters = ctl->iters_done;
  s.applies = ctl->applies_done;
  s.jacobi = ctl->jacobi_done;
  s.extrap_n = ctl->extrap_done;
  s.unconv_n = ctl->unconv_done;
  s.fvalid = ctl->fvalid;
  s.pxvalid = ctl->pxvalid;
  s.polish = ctl->polish;
  s.xvalid = ctl->xvalid;
  return s;
}

// The certificate with mu_{r+1} replaced by an upper bound of it (the
// deflated Lanczos bound armed for this step; +inf without one).  The top r
// Ritz values are lower bounds and L does not increase with them, so this
// bounds the exact L from above.  Lane-uniform; evaluated by every lane.
__device__ inline double cert_upper(const Cfg& cfg, const lds<double>* theta, const SolveScalars& sc, double eps,
                                   double mu_up) {
  if (!(mu_up < __builtin_inf())) return __builtin_inf();
  const int r = cfg.r;
  const double la = log(sc.alpha);
  double m = mu_up;
  for (int l = 0; l < r; ++l) m = fmax(m, theta[l] + la - sc.sigma);
  double e = exp(mu_up - m);
  for (int l = 0; l < r; ++l) e += exp(theta[l] + la - sc.sigma - m);
  return log((double)(cfg.n - r)) - log(eps) + mu_up - (m + log(e));
}

// End of the inner solve: exponentiate and normalise (Definition 1), build
// the next factored iterate (alpha', d', c') and the certificate.  theta
// (LDS) holds the sorted Ritz values of Yhat, rho their residuals.  One
// wavefront.
__device__ inline void finish_step(const Cfg& cfg, gbl<Ctl>* ctl, const lds<double>* theta, const lds<double>* rho,
                                   double resid_max, int sweeps, int converged, int resolved, double margin,
                                   double eps, const SolveScalars& sc, int lane, double& d_out, double& c_out,
                                   double& alpha_out, int& halt_out) {
  const int r = cfg.r;
  const double n = (double)cfg.n;
  const double alpha = sc.alpha, sigma = sc.sigma, solve_tol = sc.solve_tol;
  const int64_t t = sc.t;
  const double la = log(alpha);
  const double mu = (lane <= r) ? theta[lane] + la - sigma : -__builtin_inf();  // eigenvalues of M_t
  const double m = wave_max(mu);
  const double e = (lane <= r) ? exp(mu - m) : 0.0;
  const double sr = wave_sum(lane < r ? e : 0.0);
  const double sr1 = wave_sum(e);
  const double lse_r = m + log(sr);    // log a_t
  const double lse_r1 = m + log(sr1);  // log b^{r+1}_t
  const double mu_r1 = lane_f64(mu, r);
  const double mu_r = lane_f64(mu, r - 1);
  const double alpha_n = eps / (n - r);
  const double l1e = log1p(-eps);
  const double la_n = log(alpha_n);
  bool ok = true;
  double dl = 0.0, cl = 0.0;
  if (lane < r) {
    const double lt = mu - lse_r;              // log lambda~_l = mu_l - log a_t
    dl = (1.0 - eps) * exp(lt) - alpha_n;
    cl = l1e + lt - la_n;                      // log((1-eps) lambda~_l) - log(alpha')
    ok = isfinite(dl) && isfinite(cl);
  }
  if (lane < KMAX) {
    ctl->d[lane] = dl;
    ctl->c[lane] = cl;
  }
  d_out = dl;
  c_out = cl;
  alpha_out = alpha_n;
  const bool all_ok = wave_min(ok ? 1.0 : 0.0) > 0.5 && isfinite(lse_r1);
  halt_out = all_ok ? 0 : 1;
  if (lane == 0) {
    ctl->alpha = alpha_n;
    const double L = log(n - r) - log(eps) + mu_r1 - lse_r1;
    gbl<Info>& in = ctl->info;
    in.t = t;
    in.eps_t = eps;
    in.cert_L = L;
    in.cert_bound = fmax(2.0 * eps, L);
    // L from the Ritz values is a lower bound of the exact L; upper bounds:
    // L + margin with a resolved (r+1)-th pair, and L with mu_{r+1} replaced
    // by the deflated bound (when armed for this step); claims use the lower
    const double mu_up = fmin(resolved ? mu_r1 + margin : __builtin_inf(), sc.up_bound());
    const double L_up = cert_upper(cfg, theta, sc, eps, mu_up);
    in.cert_holds = (L_up <= 2.0 * eps) ? 1 : 0;
    in.cert_resolved = resolved;
    in.cert_L_up = L_up;
    in.mu_r1_up = mu_up;
    in.inner_iters = sweeps;
    in.ritz_gap = mu_r - mu_r1;
    in.resid_max = resid_max;
    in.resid_r1 = margin;
    in.mu_r1 = mu_r1;
    in.sigma = sigma;
    in.converged = converged;
    in.f = sc.fvalid ? sc.f : __builtin_nan("");
    if (!all_ok) ctl->status = 4;  // MEG_ERR_NUMERIC
    if (solve_tol > 0.0 && fmax(2.0 * eps, L_up) <= solve_tol) {
      ctl->stop = 1;
      halt_out = 1;  // lane 0's value is the one used
    }
  }
}

// small_sweep's outcome, the tag of the barrier it ends: the step ended
// (X_{t+1} and the next step's scalars are set); its next warm start is this
// sweep's output block (extrapolated end; otherwise its input block); the
// team stops here (a failure, a met stopping rule or a pause; ctl says which).
constexpr int kSweepEnded = 1, kSweepExtrap = 2, kSweepHalt = 4;

// One Rayleigh-Ritz / orthonormalisation step.  `sums` (LDS or global) holds the
// reduced record of PartRec: C = Zin^T Zout, G = Zout^T Zout (triangle),
// P = V^T Zout (r rows), where Zout = Yhat Q and Q = Zin W is orthonormal.
// Sets the next sweep's W and PW = V^T Q', or ends the step: the Ritz basis
// Zin (W S) becomes the next warm start (B, Wb) = (Zin, W S), advances t and
// sets the next step's shift and coefficients.  Counts the apply (and the
// Jacobi sweeps) in ctl.  `grad`: this sweep formed the masked gradient (its
// objective sums are in the record).  Returns 0 when another sweep follows,
// else the kSweep* bits of the outcome (uniform over the workgroup).
// Called by every thread of the workgroup (tid); the work runs on two
// wavefronts, wave-synchronously within each: wavefront 0 solves, wavefront
// 1 meanwhile forms eps_t and, when the step ends here, the new iterate and
// its certificate while wavefront 0 forms the next basis.  `scr` (LDS)
// needs 5 * KB * (KB + 1) + 12 * KB doubles.
template <int KB, typename SP>
__device__ __noinline__ int small_sweep(const lds<Cfg>* cfg_l, gbl<Ctl>* ctl, SP sums, lds<double>* scr,
                                         int sweep, int in_buf, int out_buf, bool grad, int tid,
                                         gbl<long long>* ts) {
  const Cfg& cfg = *(const Cfg*)cfg_l;  // LDS: its fields are read without a memory round trip
  constexpr int LD = KB + 1;
  constexpr int MS = KB * LD;
  const int lane = tid & 63, wave = tid >> 6;
  lds<double>* A = scr;            // T, then diagonalised
  lds<double>* S = scr + MS;       // Ritz vectors (unsorted)
  lds<double>* B1 = scr + 2 * MS;  // W, then sorted S
  lds<double>* B2 = scr + 3 * MS;  // C, then G S, then P S
  lds<double>* B3 = scr + 4 * MS;  // G, then Ghat = S^T G S
  lds<double>* vec = scr + 5 * MS; // 12 * KB
  lds<double>* theta = vec;
  lds<double>* rho = vec + KB;
  lds<double>* jrot = vec + 2 * KB;  // 2 * KB: rotations of a Jacobi round (KB > 16)
  lds<double>* rdiag = vec + 4 * KB;  // reciprocal diagonal of a Cholesky factor
  lds<int>* perm = reinterpret_cast<lds<int>*>(vec + 6 * KB);
  lds<double>* xch = vec + 8 * KB;   // 4 * KB: what the two wavefronts exchange
  const int r = cfg.r;
  using PR = PartRec<KB>;
  const int fo = PR::f_off(r);

  if (sweep < cfg.rr_from && sweep < cfg.max_inner) {
    if (wave == 0) {
      // early sweep of a warm-started step: orthonormalise only,
      // Q' = Zout R^{-1} with Zout^T Zout = R^T R;  PW' = V^T Zout R^{-1}
      // every global read issued before any is used (one round trip)
      const int64_t applies = ctl->applies_done;
      const double fs = sums[fo], px2 = sums[fo + 1];
      constexpr int IT = KB * KB / 64;
      double gv[IT], pv[IT];
#pragma unroll
      for (int u = 0; u < IT; ++u) {
        const int e = lane + 64 * u, i = e / KB, j = e % KB;
        gv[u] = sums[PR::G_OFF + (i <= j ? PR::tri(i, j) : PR::tri(j, i))];
        pv[u] = sums[PR::P_OFF + (i < r ? e : 0)];  // P (its r rows)
      }
#pragma unroll
      for (int u = 0; u < IT; ++u) {
        const int e = lane + 64 * u, i = e / KB, j = e % KB;
        B3[i * LD + j] = gv[u];
        B1[i * LD + j] = (i < r) ? pv[u] : 0.0;
        S[i * LD + j] = (i == j) ? 1.0 : 0.0;
      }
      wsync();
      chol_apply2<KB>(B3, S, B2, rdiag, lane);  // S = R^{-1}, B1 = P R^{-1}
      store_mat<KB>(S, ctl->W, lane);
      store_mat<KB>(B1, ctl->PW, lane);
      if (lane == 0) {
        if (grad) {  // f(X_t) = 1/2 sum_Omega g^2, ||P_Omega X_t||_F
          ctl->f = 0.5 * fs;
          ctl->fvalid = 1;
          ctl->pxnorm = sqrt(px2);
          ctl->pxvalid = 1;
        }
        ctl->sweep = sweep + 1;
        ctl->applies_done = applies + 1;
        ctl->xvalid = 0;
      }
    }
    return 0;
  }

  // Rayleigh-Ritz sweep.  Both wavefronts load the step's scalars.
  SolveScalars sc{};
  if (wave < 2) {
    sc = load_scalars(cfg, ctl, lane);
    if (grad) {
      sc.f = 0.5 * sums[fo];
      sc.fvalid = 1;
      sc.pxnorm = sqrt(sums[fo + 1]);
      sc.pxvalid = 1;
    }
  }
  if (wave == 1 && lane == 0) xch[0] = eps_at(cfg, sc.t);
  // wavefront 0's state across the sections below
  constexpr int WE = KB * KB / 64;
  constexpr int PE = KB * KB / 64;
  double wreg[WE], pnew[PE], pold[PE];
  double fa = 1.0, fb = 0.0, th = 0.0, fth = 0.0, rh = 0.0, thr = 0.0, rmax = 0.0, margin = 0.0;
  double floor_est = 0.0, tol_abs = 0.0, scale = 1.0, xr = 0.0, xthr = 0.0, rr1 = 0.0, xr1 = 0.0;
  bool exact = false, finite = true, resolved = false, light = false, cert_ok = false, top_ok = false;
  bool fin = false, extrap = false, do_polish = false;
  int jsweeps = 0, polish = 0;
  const bool prof = ts != nullptr && tid == 0 && sweep == cfg.rr_from;
  if (wave == 0) {
    // W stays in registers too: the step's end forms W S from it.  All of
    // the solve's global reads are issued before any is stored.
    double cv[WE], gv[WE];
#pragma unroll
    for (int u = 0; u < WE; ++u) {
      const int e = lane + 64 * u, i = e / KB, j = e % KB;
      wreg[u] = ctl->W[e];
      cv[u] = sums[e];  // C
      gv[u] = sums[PR::G_OFF + (i <= j ? PR::tri(i, j) : PR::tri(j, i))];
    }
    // P = V^T Zout (for the next sweep's PW) and this sweep's PW = V^T Q, held
    // in registers: the first is used only if another sweep follows, the
    // second gives V_t^T V_{t+1} = PW S[:, :r] when the step ends here
#pragma unroll
    for (int m = 0; m < PE; ++m) {
      const int e = lane + 64 * m;  // < KB * KB (PE = KB * KB / 64)
      const double pn = sums[PR::P_OFF + (e < r * KB ? e : 0)];
      pnew[m] = (e < r * KB) ? pn : 0.0;
      pold[m] = ctl->PW[e];
    }
#pragma unroll
    for (int u = 0; u < WE; ++u) {
      const int e = lane + 64 * u, o = (e / KB) * LD + (e % KB);
      B1[o] = wreg[u];
      B2[o] = cv[u];
      B3[o] = gv[u];
    }
    polish = sc.polish;
    // this sweep's filter: Zout = fa Yhat Q + fb Q (Chebyshev degree 1 on
    // [0, cheb_b]; fa = 1, fb = 0 without one)
    fa = sc.cheb_b > 0.0 ? 2.0 / sc.cheb_b : 1.0;
    fb = sc.cheb_b > 0.0 ? -1.0 : 0.0;
    wsync();
    mm_tn<KB>(B1, B2, A, lane);  // W^T C = Q^T Zout = fa Q^T Yhat Q + fb I
    wsync();
    for (int e = lane; e < KB * KB; e += 64) {  // T = Q^T Yhat Q, symmetrised
      const int i = e / KB, j = e % KB;
      if (i < j) {
        const double v = 0.5 * (A[i * LD + j] + A[j * LD + i]) / fa;
        A[i * LD + j] = v;
        A[j * LD + i] = v;
      } else if (i == j) {
        A[i * LD + i] = (A[i * LD + i] - fb) / fa;
      }
    }
    wsync();
    // profiled launches: stamps of the first Rayleigh-Ritz sweep's parts
    if (prof) ts[kTsRR] = wall_clock64();
    // Off-diagonal mass left by Jacobi, relative: 1e-8 for an FP32 state
    // (below its unit roundoff 6e-8; the eigenvectors then carry errors of
    // off/gap, and the residual test sees at most 1e-8 of the scale), 1e-15
    // for FP64.  The tolerance is on squared norms.
    // (FP32 state: rotation angles from FP32 arithmetic, see jacobi_rot_f32angle)
    jsweeps = cfg.unit_round < 1e-10 ? jacobi<KB, false>(A, S, 1e-30, lane, jrot)
                                     : jacobi<KB, true>(A, S, 1e-16, lane, jrot);
    if (lane == 0) ctl->jacobi_done = sc.jacobi + jsweeps;
    if (prof) {
      ts[kTsRR + 1] = wall_clock64();
      ts[kTsRR + 4] = jsweeps;
    }
    // sort eigenvalues descending: rank of each diagonal entry, ties broken by
    // index; NaN ranks as -inf so the ranks always form a permutation (the NaN
    // itself is caught by the finiteness check below)
    if (lane < KB) {
      const double v0 = A[lane * LD + lane];
      const double v = isnan(v0) ? -__builtin_inf() : v0;
      int rank = 0;
  #pragma unroll
      for (int j = 0; j < KB; ++j) {
        const double w0 = A[j * LD + j];
        const double w = isnan(w0) ? -__builtin_inf() : w0;
        rank += (w > v || (w == v && j < lane)) ? 1 : 0;
      }
      perm[rank] = lane;
      theta[rank] = v0;
    }
    wsync();
    for (int e = lane; e < KB * KB; e += 64) {  // B1 <- sorted S
      const int i = e / KB, j = e % KB;
      B1[i * LD + j] = S[i * LD + perm[j]];
    }
    wsync();
    mm_nn<KB>(B3, B1, B2, lane);  // G S
    wsync();
    mm_tn<KB>(B1, B2, B3, lane);  // Ghat = S^T G S  (Gram of Zout S)
    wsync();
    // Ritz residuals: Zout s_i = (fa theta_i + fb) q_i + fa (Yhat q_i - theta_i q_i),
    // so ||Yhat q_i - theta_i q_i||^2 = (Ghat_ii - (fa theta_i + fb)^2) / fa^2
    th = (lane < KB) ? theta[lane] : 0.0;
    fth = fa * th + fb;
    rh = (lane < KB) ? sqrt(fmax(B3[lane * LD + lane] - fth * fth, 0.0)) / fabs(fa) : 0.0;
    if (lane < KB) {
      rho[lane] = rh;
      ctl->theta[lane] = th;
      ctl->resid[lane] = rh;
    }
    scale = fmax(fabs(lane_f64(th, 0)), 1e-300);
    // Residuals come from Ghat_ii - theta_i^2 in FP64: resolvable down to
    // ~sqrt(2^-53) of the scale; working-precision rounding sets another floor.
    floor_est = fmax(3e-8, 8.0 * cfg.unit_round) * scale;
    tol_abs = cfg.inner_tol * scale;
    thr = fmax(tol_abs, floor_est);
    // Below that floor (FP64 state) the test also needs the explicit residuals
    // ||Zout s_i - theta_i Q s_i|| of the previous sweep's pairs, which this
    // sweep's apply formed from its rows; this sweep's pairs are one power
    // step further on.  Their floor is the apply's rounding.
    exact = cfg.xres && tol_abs < floor_est;
    xthr = fmax(tol_abs, 64.0 * cfg.unit_round * scale);
    xr = (exact && sc.xvalid && lane < KB) ? sqrt(fmax(sums[PR::x_off(r) + lane], 0.0)) * sc.xscale
                                                        : __builtin_inf();
    rmax = wave_max(lane < r ? rh : 0.0);
    finite = wave_min((lane < KB) ? ((isfinite(th) && isfinite(rh)) ? 1.0 : 0.0) : 1.0) > 0.5;
    rr1 = lane_f64(rh, r);
    xr1 = lane_f64(xr, r);
  }
  __syncthreads();  // eps_t from wavefront 1
  const double eps_t = xch[0];
  if (wave == 0) {
    // A top-r pair enters X_{t+1} = alpha' I + V diag(d') V^T only through
    // d'_l v_l v_l^T: even an entirely wrong v_l moves X by at most
    // sqrt(2) |d'_l|, i.e. sqrt(2) w_l of ||X||_F with w_l = |d'_l| / max |d'|.
    // Pairs with w_l <= inner_tol / 4 therefore need no residual test (in the
    // noise bulk of M_t such pairs converge slowly and carry no weight).
    // d' follows from the Ritz values exactly as finish_step forms it.
    const double mu = (lane < r) ? th + log(sc.alpha) - sc.sigma : -__builtin_inf();
    const double mmax = wave_max(mu);
    const double ex = (lane < r) ? exp(mu - mmax) : 0.0;
    const double esum = wave_sum(ex);
    const double dl_new = (lane < r) ? (1.0 - eps_t) * ex / esum - eps_t / (double)(cfg.n - r) : 0.0;
    const double dmax = wave_max(fabs(dl_new));
    light = dmax > 0.0 && fabs(dl_new) <= 0.25 * cfg.inner_tol * dmax;
    const bool pair_ok = lane >= r || light || (rh <= thr && (!exact || xr <= xthr));
    // Certificate L_t = log(n-r) - log eps_t + mu_{r+1} - LSE(mu_1..mu_{r+1}).
    // The Ritz values are lower bounds of the eigenvalues (interlacing) and
    // dL/dmu_{r+1} = 1 - softmax_{r+1} lies in [0, 1] (dL/dmu_i <= 0, i <= r),
    // so L from the Ritz values is a lower bound of the exact L.  A Ritz value
    // is within its residual of SOME eigenvalue; inside a cluster that need not
    // be lambda_{r+1}.  The (r+1)-th pair counts as resolved when its residual
    // bound rho (the estimate, not below its floor, or the explicit residual of
    // the previous sweep's pair) meets the tolerance and is at most a quarter
    // of the gap to theta_{r+2}: the Ritz value is then isolated, and L + rho
    // bounds the exact L from above.  Only then is a certificate claimed.
    margin = fmin(fmax(rr1, floor_est), exact ? xr1 : __builtin_inf());
    const double sep = (r + 2 <= KB) ? lane_f64(th, r) - lane_f64(th, r + 1 < KB ? r + 1 : r) : 0.0;
    const double cthr = cfg.cert_tol > 0.0 ? fmax(cfg.cert_tol, exact ? 64.0 * cfg.unit_round * scale : floor_est)
                                           : (exact ? xthr : thr);
    resolved = margin <= cthr && margin <= 0.25 * sep;
    // The pair is iterated further, until resolved or max_inner, always for
    // cert_tol > 0, and for a stopping rule (meg_solve's or a server's tol)
    // while its lower bound of L could pass: otherwise the step takes no
    // sweeps for it and claims nothing while it is unresolved.
    bool pending = false;
    if (sc.solve_tol > 0.0) {  // only a stopping rule may ask for more sweeps here
      const double mu1 = (lane <= r) ? th + log(sc.alpha) - sc.sigma : -__builtin_inf();
      const double m1 = wave_max(mu1);
      const double lse1 = m1 + log(wave_sum((lane <= r) ? exp(mu1 - m1) : 0.0));
      const double L_lo = log((double)(cfg.n - r)) - log(eps_t) + lane_f64(mu1, r) - lse1;
      const double cut = fmax(2.0 * eps_t, sc.solve_tol);
      pending = !(L_lo > cut) && !(cert_upper(cfg, theta, sc, eps_t, sc.up_bound()) <= cut);
    }
    cert_ok = resolved || !(cfg.cert_tol > 0.0 || pending);
    top_ok = wave_min(pair_ok ? 1.0 : 0.0) > 0.5;
    bool conv = top_ok && cert_ok;
    // tolerance below the resolvable floor without explicit residuals (FP32
    // state): two more sweeps once it is reached
    if (conv && !cfg.xres && tol_abs < floor_est && polish < 2) {
      do_polish = true;
      conv = false;
    }
    wsync();
    if (prof) ts[kTsRR + 2] = wall_clock64();
    fin = !finite || (conv && sweep >= cfg.min_inner) || sweep >= cfg.max_inner;
    if (!finite && lane == 0) {
      ctl->status = 4;  // MEG_ERR_NUMERIC
      ctl->stop = 1;
      ctl->done = 1;
      ctl->applies_done = sc.applies + 1;
    }
    // Extrapolated end (FP32 forms): when every top pair's residual, times the
    // power step's contraction theta_k / theta_i (at most 0.05: a gap the
    // prediction is reliable across) and a safety factor 2, meets the
    // tolerance, the block Zout S after one more power step is accepted
    // without a further sweep to test it; the Ritz values of this sweep are
    // kept (their error is second order in the residuals).
    if (!fin && cfg.extrap && !exact && cert_ok && sweep >= cfg.min_inner) {
      // contraction of the power step just taken: the unwanted spectrum,
      // taken to lie in [0, theta_k], maps to at most max(|fb|, |fa theta_k + fb|)
      const double thk = fmax(fabs(fb), fabs(fa * lane_f64(th, KB - 1) + fb));
      const double ratio = (lane < r) ? thk / fmax(fabs(fth), 1e-300) : 0.0;
      const bool ok = lane >= r || light || (ratio <= 0.05 && 2.0 * ratio * rh <= thr);
      extrap = wave_min(ok ? 1.0 : 0.0) > 0.5;
    }
    const int code = !finite ? 4 : (fin ? 1 : (extrap ? 2 : 0));
    if (lane == 0) {
      xch[1] = code;
      xch[2] = rmax;
      xch[3] = (extrap || (top_ok && (resolved || !(cfg.cert_tol > 0.0)))) ? 1.0 : 0.0;  // converged
      xch[4] = resolved ? 1.0 : 0.0;
      xch[5] = margin;
      if (grad) {
        ctl->f = sc.f;
        ctl->fvalid = 1;
        ctl->pxnorm = sc.pxnorm;
        ctl->pxvalid = 1;
      }
    }
  }
  __syncthreads();  // the decision
  const int code = (int)xch[1];
  if (code == 4) return kSweepHalt;
  if (code != 0) {
    // the step ends here: wavefront 1 exponentiates and normalises and
    // forms the certificate, wavefront 0 the next basis
    if (wave == 1) {
      double d_new, c_new, a_new;
      int halt;
      finish_step(cfg, ctl, theta, rho, xch[2], sweep, (int)xch[3], (int)xch[4], xch[5], eps_t, sc, lane, d_new,
                  c_new, a_new, halt);
      if (lane < KB) {
        xch[8 + lane] = d_new;
        xch[8 + KB + lane] = c_new;
      }
      if (lane == 0) {
        xch[8 + 2 * KB] = a_new;
        xch[8 + 2 * KB + 1] = halt;
      }
    }
    lds<double>* Cm = B3;
    if (wave == 0) {
      extrap = code == 2;
      // The next warm start (B, Wb) and C = V_t^T V_{t+1} (first r x r) for
      // ||X_{t+1} - X_t||_F:
      //  - ended here: the Ritz vectors of span(Q), Q S = Zin (W S); C = PW S;
      //  - extrapolated: Zout S R^{-1} (Cholesky QR, S^T G S = R^T R), whose first
      //    r columns span the power step of the top pairs; C = P S R^{-1}.
      // The next step's first sweep uses W = Wb and PW = V^T Q = [I_r 0].
      lds<double>* Wn;  // the next W = Wb
      if (extrap) {
  #pragma unroll
        for (int m = 0; m < PE; ++m) {
          const int e = lane + 64 * m;
          if (e < KB * KB) S[(e / KB) * LD + (e % KB)] = pnew[m];
        }
        wsync();
        mm_nn<KB>(S, B1, B2, lane);  // B2 = P S
        wsync();
        chol_apply2<KB>(B3, B1, A, rdiag, lane);  // B1 = S R^{-1}, B2 = P S R^{-1}
        Wn = B1;
        Cm = B2;
      } else {
  #pragma unroll
        for (int u = 0; u < WE; ++u) {
          const int e = lane + 64 * u;
          B2[(e / KB) * LD + (e % KB)] = wreg[u];
        }
  #pragma unroll
        for (int m = 0; m < PE; ++m) {
          const int e = lane + 64 * m;
          if (e < KB * KB) S[(e / KB) * LD + (e % KB)] = pold[m];
        }
        wsync();
        mm_nn<KB>(B2, B1, A, lane);  // A = W S
        mm_nn<KB>(S, B1, B3, lane);  // PW S
        wsync();
        Wn = A;
        Cm = B3;
      }
      store_mat<KB>(Wn, ctl->Wb, lane);
      store_mat<KB>(Wn, ctl->W, lane);
      for (int e = lane; e < KB * KB; e += 64) ctl->PW[e] = (e / KB == e % KB && e / KB < r) ? 1.0 : 0.0;
    }
    __syncthreads();  // the new iterate from wavefront 1
    if (wave == 0) {
      const double a_old = sc.alpha;
      const double d_old = sc.dl;
      const double d_new = (lane < KB) ? xch[8 + lane] : 0.0;
      const double c_new = (lane < KB) ? xch[8 + KB + lane] : 0.0;
      const double a_new = xch[8 + 2 * KB];
      // ||X_{t+1} - X_t||_F from the factored forms (V orthonormal):
      //   n da^2 + 2 da (sum d_t - sum d_{t+1}) + |d_t|^2 + |d_{t+1}|^2
      //   - 2 sum_ab d_t,a d_{t+1},b C_ab^2
      lds<double>* dd = vec + 2 * KB;  // the Jacobi rotations' area: d_t, then d_{t+1}
      if (lane < KB) {
        dd[lane] = d_old;
        dd[KB + lane] = d_new;
      }
      wsync();
      double cross = 0.0;
      for (int e = lane; e < r * r; e += 64) {
        const int a = e / r, b = e % r;
        const double c = Cm[a * LD + b];
        cross += dd[a] * dd[KB + b] * c * c;
      }
      cross = wave_sum(cross);
      const double sd = wave_sum(d_old - d_new);
      const double s2 = wave_sum(d_old * d_old + d_new * d_new);
      const double da = a_old - a_new;
      const double dx2 = (double)cfg.n * da * da + 2.0 * da * sd + s2 - 2.0 * cross;
      const double dxnorm = sqrt(fmax(dx2, 0.0));
      // step t + 1 begins: its counters, then its shift and coefficients from
      // the values in registers
      if (lane == 0) {
        ctl->dxnorm = dxnorm;
        ctl->src = extrap ? out_buf : in_buf;
        ctl->t = sc.t + 1;
        ctl->iters_done = sc.iters + 1;
        ctl->applies_done = sc.applies + 1;
        ctl->fvalid = 0;
        ctl->done = 0;
        ctl->sweep = 1;
        ctl->polish = 0;
        ctl->xvalid = 0;
        ctl->extrap_done = sc.extrap_n + (extrap ? 1 : 0);
        ctl->unconv_done = sc.unconv_n + ((extrap || top_ok) ? 0 : 1);
      }
      const double la = log(sc.alpha);
      const double mu_1 = theta[0] + la - sc.sigma, mu_k = theta[KB - 1] + la - sc.sigma;
      if (lane == 0) {
        ctl->mu_1 = mu_1;
        ctl->mu_k = mu_k;
        ctl->mu_valid = 1;
      }
      if (cfg.kind != QUADMEAS) {  // the minibatch bound is set inside the next step's first sweep
        const double gmax =
            grad_bound(cfg, a_new, d_new, sc.op_lmin, sc.op_lmax, sc.pxvalid, sc.pxnorm, dxnorm, lane);
        setup_step_v(cfg, ctl, gmax, a_new, d_new, c_new, mu_1, mu_k, 1, lane);
      }
      if (prof) ts[kTsRR + 3] = wall_clock64();
    }
    return kSweepEnded | (code == 2 ? kSweepExtrap : 0) | (xch[8 + 2 * KB + 1] != 0.0 ? kSweepHalt : 0);
  }
  if (wave == 0) {
    if (cfg.xres) {
      // for the next sweep's explicit residuals: S and W S Theta
  #pragma unroll
      for (int u = 0; u < WE; ++u) {
        const int e = lane + 64 * u;
        B2[(e / KB) * LD + (e % KB)] = wreg[u];
      }
      wsync();
      mm_nn<KB>(B2, B1, A, lane);
      wsync();
      for (int e = lane; e < KB * KB; e += 64) {
        const int i = e / KB, j = e % KB;
        ctl->XS[e] = B1[i * LD + j];
        ctl->XWT[e] = A[i * LD + j] * (fa * theta[j] + fb);
      }
      if (lane == 0) {
        ctl->xvalid = 1;
        ctl->xscale = 1.0 / fabs(fa);
      }
      wsync();
    }
    // Next basis Q' = Zout S R^{-1} with Ghat = R^T R (Cholesky QR, FP64) and
    // PW' = V^T Q' = P S R^{-1}
  #pragma unroll
    for (int m = 0; m < PE; ++m) {
      const int e = lane + 64 * m;
      if (e < KB * KB) S[(e / KB) * LD + (e % KB)] = pnew[m];
    }
    wsync();
    mm_nn<KB>(S, B1, B2, lane);  // B2 = P S
    wsync();
    chol_apply2<KB>(B3, B1, A, rdiag, lane);  // B1 = W' = S R^{-1}, B2 = PW' = P S R^{-1}
    store_mat<KB>(B1, ctl->W, lane);
    store_mat<KB>(B2, ctl->PW, lane);
    if (lane == 0) {
      ctl->sweep = sweep + 1;
      ctl->applies_done = sc.applies + 1;
      if (do_polish) ctl->polish = polish + 1;
      // the next sweep's Chebyshev interval: [0, theta_k] of this one
      const double b = theta[KB - 1];
      ctl->cheb_b = (cfg.cheb && b > 1e-3 * theta[0] && b < 0.5 * theta[0]) ? b : 0.0;
    }
    if (prof) ts[kTsRR + 3] = wall_clock64();
  }
  return 0;
}

// Orthonormalising transform of a fresh basis B with Gram H = B^T B:
// Wb = W = R^{-1} (H = R^T R), so Q = B Wb is orthonormal and V = Q[:, :r];
// PW = V^T Q = [I_r 0].  One wavefront.
template <int KB>
__device__ __noinline__ void basis_setup(const Cfg& cfg, gbl<Ctl>* ctl, const gbl<double>* gram, lds<double>* scr,
                                         int lane) {
  constexpr int MS = KB * (KB + 1);
  constexpr int LD = KB + 1;
  lds<double>* A = scr;
  lds<double>* Rinv = scr + MS;
  lds<double>* R = scr + 2 * MS;
  lds<double>* rdiag = scr + 3 * MS;
  load_mat<KB>(gram, A, lane);
  for (int e = lane; e < KB * KB; e += 64) Rinv[(e / KB) * LD + (e % KB)] = (e / KB == e % KB) ? 1.0 : 0.0;
  wsync();
  chol_factor<KB>(A, R, rdiag, lane);
  rsolve<KB>(Rinv, Rinv, R, rdiag, KB, lane);
  store_mat<KB>(Rinv, ctl->W, lane);
  store_mat<KB>(Rinv, ctl->Wb, lane);
  for (int e = lane; e < KB * KB; e += 64) ctl->PW[e] = (e / KB == e % KB && e / KB < cfg.r) ? 1.0 : 0.0;
  if (lane == 0) {
    ctl->done = 0;
    ctl->sweep = 1;
    ctl->polish = 0;
    ctl->xvalid = 0;
  }
}

}  // namespace meg
