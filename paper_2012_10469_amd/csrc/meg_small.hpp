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

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// C = A^T B (all KB x KB, LDS stride KB + 1)
template <int KB>
__device__ __forceinline__ void mm_tn(const double* A, const double* B, double* C, int lane) {
  constexpr int LD = KB + 1;
  for (int e = lane; e < KB * KB; e += 64) {
    const int i = e / KB, j = e % KB;
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < KB; ++l) s += A[l * LD + i] * B[l * LD + j];
    C[i * LD + j] = s;
  }
}

// C = A B
template <int KB>
__device__ __forceinline__ void mm_nn(const double* A, const double* B, double* C, int lane) {
  constexpr int LD = KB + 1;
  for (int e = lane; e < KB * KB; e += 64) {
    const int i = e / KB, j = e % KB;
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < KB; ++l) s += A[i * LD + l] * B[l * LD + j];
    C[i * LD + j] = s;
  }
}

// dense KB x KB (stride KB, global or LDS) <-> LDS stride KB + 1; the loops
// have compile-time trip counts so all loads are issued before any is used
template <int KB>
__device__ __forceinline__ void load_mat(const double* src, double* dst, int lane) {
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

template <int KB>
__device__ __forceinline__ void store_mat(const double* src, double* dst, int lane) {
#pragma unroll
  for (int u = 0; u < KB * KB / 64; ++u) {
    const int e = lane + 64 * u;
    dst[e] = src[(e / KB) * (KB + 1) + (e % KB)];
  }
}

// dst[e] = src[e], e < KB * KB (global to global), all loads in flight
template <int KB>
__device__ __forceinline__ void copy_mat(const double* src, double* dst, int lane) {
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

// Cyclic parallel Jacobi (round-robin ordering) for symmetric A in LDS.
// On return A is (numerically) diagonal and A_in = S diag(A) S^T.  Stops
// when the off-diagonal mass is below off2_tol of the total (squared norms).
// Each round applies KB/2 disjoint rotations: lane m < KB/2 computes rotation
// m (c^2 + s^2 = 1 to rounding, so S stays orthogonal however approximate
// the angle), then every lane updates whole 2 x 2 blocks J_m^T A_{mm'} J_m'
// and pairs of S columns, reading the parameters by shuffles.
template <int KB>
__device__ __noinline__ void jacobi(double* A, double* S, double off2_tol, int lane) {
  constexpr int LD = KB + 1;
  constexpr int NP = KB / 2;
  static_assert((NP * NP) % 64 == 0 && (KB * NP) % 64 == 0, "block counts must fill the wavefront");
  constexpr int BPL = NP * NP / 64;  // 2 x 2 blocks per lane
  constexpr int SPL = KB * NP / 64;  // S column pairs per lane
  for (int e = lane; e < KB * KB; e += 64) S[(e / KB) * LD + (e % KB)] = (e / KB == e % KB) ? 1.0 : 0.0;
  wsync();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < KB * KB; e += 64) {
      const double v = A[(e / KB) * LD + (e % KB)];
      if (e / KB == e % KB) dia += v * v; else off += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if (!(off > off2_tol * (off + dia))) break;  // also exits on NaN
    for (int round = 0; round < KB - 1; ++round) {
      int p = 0, q = 1;
      double c = 1.0, s = 0.0;
      if (lane < NP) {
        // circle method: slot 0 fixed, slots 1..KB-1 rotate by `round`
        const int a = lane, b = KB - 1 - lane;
        const int pa = (a == 0) ? 0 : 1 + ((a - 1 + round) % (KB - 1));
        const int pb = 1 + ((b - 1 + round) % (KB - 1));
        p = min(pa, pb);
        q = max(pa, pb);
        const double apq = A[p * LD + q], app = A[p * LD + p], aqq = A[q * LD + q];
        if (apq * apq > 1e-36 * fabs(app * aqq) && fabs(apq) > 1e-300) {
          // tangent of the rotation angle: t = sign(tau) / (|tau| + sqrt(1 + tau^2))
          const double tau = 0.5 * (aqq - app) * rcp_nr(apq);
          double t;
          if (fabs(tau) > 1e100) {
            t = 0.5 * rcp_nr(tau);
          } else {
            const double h = 1.0 + tau * tau;
            t = rcp_nr(fabs(tau) + h * rsqrt_nr(h));
            t = (tau >= 0.0) ? t : -t;
          }
          c = rsqrt_nr(1.0 + t * t);
          s = t * c;
        }
      }
#pragma unroll
      for (int bi = 0; bi < BPL; ++bi) {
        const int blk = lane + 64 * bi;
        const int m1 = blk / NP, m2 = blk % NP;
        const int p1 = __shfl(p, m1, 64), q1 = __shfl(q, m1, 64);
        const int p2 = __shfl(p, m2, 64), q2 = __shfl(q, m2, 64);
        const double c1 = __shfl(c, m1, 64), s1 = __shfl(s, m1, 64);
        const double c2 = __shfl(c, m2, 64), s2 = __shfl(s, m2, 64);
        const double a = A[p1 * LD + p2], b = A[p1 * LD + q2], cc = A[q1 * LD + p2], d = A[q1 * LD + q2];
        const double ra = c1 * a - s1 * cc, rb = c1 * b - s1 * d;  // rows: J1^T
        const double rc = s1 * a + c1 * cc, rd = s1 * b + c1 * d;
        A[p1 * LD + p2] = c2 * ra - s2 * rb;                       // columns: J2
        A[p1 * LD + q2] = s2 * ra + c2 * rb;
        A[q1 * LD + p2] = c2 * rc - s2 * rd;
        A[q1 * LD + q2] = s2 * rc + c2 * rd;
      }
#pragma unroll
      for (int si = 0; si < SPL; ++si) {
        const int pr = lane + 64 * si;
        const int i = pr / NP, m = pr % NP;
        const int pp = __shfl(p, m, 64), qq = __shfl(q, m, 64);
        const double cm = __shfl(c, m, 64), sm = __shfl(s, m, 64);
        const double x = S[i * LD + pp], y = S[i * LD + qq];
        S[i * LD + pp] = cm * x - sm * y;
        S[i * LD + qq] = sm * x + cm * y;
      }
      wsync();
    }
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
// upper triangle read), then Rinv = R^{-1} (upper, LDS).  Lane c holds
// column c in registers; every value another lane needs is a readlane of a
// compile-time lane index, so the factorisation touches no memory.  Tiny
// pivots are floored to keep R invertible.
template <int KB>
__device__ __noinline__ void chol_inv(const double* A, double* Rinv, int lane) {
  constexpr int LD = KB + 1;
  double a[KB];  // column `lane` of A, overwritten by column `lane` of R
#pragma unroll
  for (int i = 0; i < KB; ++i) a[i] = (lane < KB && i <= lane) ? A[i * LD + lane] : 0.0;
  const double scale = wave_max(lane < KB ? A[lane * LD + lane] : 0.0);
  const double floor_piv = fmax(scale, 1e-300) * 1e-28;
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    double dj = readlane_d(a[j], j);
    if (!(dj > floor_piv)) dj = floor_piv;
    const double rinv = rsqrt_nr(dj);
    // row j of R: R_jj = sqrt(dj) (lane j), R_jc = A_jc / R_jj (lanes c > j)
    a[j] = (lane == j) ? dj * rinv : a[j] * rinv;
#pragma unroll
    for (int i = j + 1; i < KB; ++i) {
      const double rji = readlane_d(a[j], i);  // R_ji, held by lane i
      if (lane >= i) a[i] -= rji * a[j];      // A_ic -= R_ji R_jc, i <= c
    }
  }
  // R X = I, column `lane` of X by back substitution; R_il is a[i] of lane l
  double x[KB];
#pragma unroll
  for (int i = KB - 1; i >= 0; --i) {
    double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int l = i + 1; l < KB; ++l) s -= readlane_d(a[i], l) * x[l];
    x[i] = (i > lane) ? 0.0 : s * rcp_nr(readlane_d(a[i], i));
  }
  if (lane < KB) {
#pragma unroll
    for (int i = 0; i < KB; ++i) Rinv[i * LD + lane] = x[i];
  }
  wsync();
}

// Per-step operator coefficients: Yhat = V diag(ceff) V^T + opscale*Op + sdiag*I
// equals M_t - log(alpha) I + sigma I.  gmax is an upper bound of
// lambda_max(grad f(X_t)); by Weyl's inequality
//   lambda_min(V diag(c) V^T - eta G) >= min(0, min c) - eta gmax,
// so sigma = eta gmax - min(0, min c) (+ a small margin) makes Yhat >= 0 and
// subspace iteration targets the algebraically largest eigenvalues.  A tight
// gmax matters: the unwanted spectrum then starts near 0, which is what makes
// the (r+1)-th pair converge.  One wavefront (all 64 lanes call it).
__device__ inline void setup_step(const Cfg& cfg, Ctl* ctl, double gmax, int lane) {
  const int r = cfg.r;
  const bool act = lane < r;
  const double cl = act ? ctl->c[lane] : 0.0;
  const double dl = act ? ctl->d[lane] : 0.0;
  const double cmin = wave_min(act ? fmin(cl, 0.0) : 0.0);
  const double cmax = wave_max(act ? fmax(cl, 0.0) : 0.0);
  const double base = cfg.eta * gmax - cmin;
  const double sigma = base + 1e-3 * (fabs(base) + cmax) + 1e-30;
  const double alpha = ctl->alpha;
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
    ctl->info.t = ctl->t;
    ctl->info.sigma = sigma;
    ctl->info.f = ctl->fvalid ? ctl->f : __builtin_nan("");
  }
}

// End of the inner solve: exponentiate and normalise (Definition 1), build
// the next factored iterate (alpha', d', c') and the certificate.  theta
// (LDS) holds the sorted Ritz values of Yhat, rho their residuals.  One
// wavefront.
__device__ inline void finish_step(const Cfg& cfg, Ctl* ctl, const double* theta, const double* rho,
                                   double resid_max, int sweeps, int converged, int lane) {
  const int r = cfg.r;
  const double n = (double)cfg.n;
  const double alpha = ctl->alpha, sigma = ctl->sigma, solve_tol = ctl->solve_tol;
  const int64_t t = ctl->t;
  const double la = log(alpha);
  const double mu = (lane <= r) ? theta[lane] + la - sigma : -__builtin_inf();  // eigenvalues of M_t
  const double m = wave_max(mu);
  const double e = (lane <= r) ? exp(mu - m) : 0.0;
  const double sr = wave_sum(lane < r ? e : 0.0);
  const double sr1 = wave_sum(e);
  const double lse_r = m + log(sr);    // log a_t
  const double lse_r1 = m + log(sr1);  // log b^{r+1}_t
  const double mu_r1 = __shfl(mu, r, 64);
  const double mu_r = __shfl(mu, r - 1, 64);
  const double eps = eps_at(cfg, t);
  const double alpha_n = eps / (n - r);
  const double l1e = log1p(-eps);
  const double la_n = log(alpha_n);
  bool ok = true;
  if (lane < KMAX) {
    double dl = 0.0, cl = 0.0;
    if (lane < r) {
      const double lt = mu - lse_r;              // log lambda~_l = mu_l - log a_t
      dl = (1.0 - eps) * exp(lt) - alpha_n;
      cl = l1e + lt - la_n;                      // log((1-eps) lambda~_l) - log(alpha')
      ok = isfinite(dl) && isfinite(cl);
    }
    ctl->d[lane] = dl;
    ctl->c[lane] = cl;
  }
  const bool all_ok = wave_min(ok ? 1.0 : 0.0) > 0.5 && isfinite(lse_r1);
  if (lane == 0) {
    ctl->alpha = alpha_n;
    const double L = log(n - r) - log(eps) + mu_r1 - lse_r1;
    Info& in = ctl->info;
    in.t = t;
    in.eps_t = eps;
    in.cert_L = L;
    in.cert_bound = fmax(2.0 * eps, L);
    in.cert_holds = (L <= 2.0 * eps) ? 1 : 0;
    in.inner_iters = sweeps;
    in.ritz_gap = mu_r - mu_r1;
    in.resid_max = resid_max;
    in.resid_r1 = rho[r];
    in.mu_r1 = mu_r1;
    in.sigma = sigma;
    in.converged = converged;
    if (!all_ok) ctl->status = 4;  // MEG_ERR_NUMERIC
    if (solve_tol > 0.0 && in.cert_bound <= solve_tol) ctl->stop = 1;
  }
}

// One Rayleigh-Ritz / orthonormalisation step.  `sums` (global) holds, stride KB:
//   C = Zin^T Zout, G = Zout^T Zout, P = V^T Zout (first r rows)
// where Zout = Yhat Q and Q = Zin W is orthonormal.  One wavefront (lanes
// 0..63).  `scr` (LDS) needs 5 * KB * (KB + 1) + 8 * KB doubles.
template <int KB>
__device__ __noinline__ void small_sweep(const Cfg& cfg, Ctl* ctl, const double* sums, double* scr, int sweep,
                                         int in_buf, int lane) {
  constexpr int LD = KB + 1;
  constexpr int MS = KB * LD;
  double* A = scr;            // T, then diagonalised
  double* S = scr + MS;       // Ritz vectors (unsorted)
  double* B1 = scr + 2 * MS;  // W, then sorted S
  double* B2 = scr + 3 * MS;  // C, then G S, then Rinv
  double* B3 = scr + 4 * MS;  // G, then Ghat = S^T G S
  double* vec = scr + 5 * MS; // 8 * KB
  double* theta = vec;
  double* rho = vec + KB;
  int* perm = reinterpret_cast<int*>(vec + 6 * KB);
  const int r = cfg.r;

  if (sweep < cfg.rr_from && sweep < cfg.max_inner) {
    // early sweep of a warm-started step: orthonormalise only,
    // Q' = Zout R^{-1} with Zout^T Zout = R^T R
    load_mat<KB>(sums + KB * KB, B3, lane);
    copy_mat<KB>(sums + 2 * KB * KB, ctl->Pin, lane);  // V^T Zout
    wsync();
    chol_inv<KB>(B3, B2, lane);
    store_mat<KB>(B2, ctl->W, lane);
    if (lane == 0) ctl->sweep = sweep + 1;
    return;
  }

  load_mat<KB>(ctl->W, B1, lane);
  load_mat<KB>(sums, B2, lane);
  load_mat<KB>(sums + KB * KB, B3, lane);
  copy_mat<KB>(sums + 2 * KB * KB, ctl->Pin, lane);  // V^T Zout (next sweep)
  const int polish = ctl->polish;
  wsync();
  mm_tn<KB>(B1, B2, A, lane);  // T = W^T C = Q^T Yhat Q
  wsync();
  for (int e = lane; e < KB * KB; e += 64) {  // symmetrise
    const int i = e / KB, j = e % KB;
    if (i < j) {
      const double v = 0.5 * (A[i * LD + j] + A[j * LD + i]);
      A[i * LD + j] = v;
      A[j * LD + i] = v;
    }
  }
  wsync();
  // eigenvector accuracy needed: rounding level of the working precision
  jacobi<KB>(A, S, cfg.unit_round < 1e-10 ? 1e-30 : 1e-22, lane);
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
  // Ritz residuals ||Yhat q s_i - theta_i q s_i||^2 = Ghat_ii - theta_i^2
  const double th = (lane < KB) ? theta[lane] : 0.0;
  const double rh = (lane < KB) ? sqrt(fmax(B3[lane * LD + lane] - th * th, 0.0)) : 0.0;
  if (lane < KB) {
    rho[lane] = rh;
    ctl->theta[lane] = th;
    ctl->resid[lane] = rh;
  }
  const double scale = fmax(fabs(__shfl(th, 0, 64)), 1e-300);
  // Residuals come from Ghat_ii - theta_i^2 in FP64: resolvable down to
  // ~sqrt(2^-53) of the scale; working-precision rounding sets another floor.
  const double floor_est = fmax(3e-8, 8.0 * cfg.unit_round) * scale;
  const double thr = fmax(cfg.inner_tol * scale, floor_est);
  const double rmax = wave_max(lane < r ? rh : 0.0);
  const bool finite = wave_min((lane < KB) ? ((isfinite(th) && isfinite(rh)) ? 1.0 : 0.0) : 1.0) > 0.5;
  const double rr1 = __shfl(rh, r, 64);
  const bool cert_ok = !(cfg.cert_tol > 0.0) || rr1 <= fmax(cfg.cert_tol, floor_est);
  bool conv = rmax <= thr && cert_ok;
  bool do_polish = false;
  // tolerance below the resolvable floor: two more sweeps once it is reached
  if (conv && cfg.inner_tol * scale < floor_est && polish < 2) {
    do_polish = true;
    conv = false;
  }
  wsync();
  const bool fin = !finite || (conv && sweep >= cfg.min_inner) || sweep >= cfg.max_inner;
  if (!finite) {
    if (lane == 0) {
      ctl->status = 4;  // MEG_ERR_NUMERIC
      ctl->stop = 1;
      ctl->done = 1;
    }
    return;
  }
  if (fin) {
    finish_step(cfg, ctl, theta, rho, rmax, sweep, conv ? 1 : 0, lane);
    // Ritz vectors of span(Q): Q S = Zin (W S)
    load_mat<KB>(ctl->W, B2, lane);
    wsync();
    mm_nn<KB>(B2, B1, A, lane);
    wsync();
    store_mat<KB>(A, ctl->Wfin, lane);
    if (lane == 0) {
      ctl->src = in_buf;
      ctl->done = 1;
    }
    return;
  }
  // Next basis Q' = Zout S R^{-1} with Ghat = R^T R (Cholesky QR, FP64)
  chol_inv<KB>(B3, B2, lane);
  mm_nn<KB>(B1, B2, A, lane);  // W' = S R^{-1}
  wsync();
  store_mat<KB>(A, ctl->W, lane);
  if (lane == 0) {
    ctl->sweep = sweep + 1;
    if (do_polish) ctl->polish = polish + 1;
  }
}

// Orthonormalising transform of a fresh basis Qw with Gram H = Qw^T Qw:
// W = R^{-1} (H = R^T R), Pin = V^T Qw = H[0:r, :].  One wavefront.
template <int KB>
__device__ __noinline__ void basis_setup(const Cfg& cfg, Ctl* ctl, const double* gram, double* scr, int lane) {
  constexpr int MS = KB * (KB + 1);
  double* A = scr;
  double* Rinv = scr + MS;
  copy_mat<KB>(gram, ctl->Pin, lane);
  load_mat<KB>(gram, A, lane);
  wsync();
  chol_inv<KB>(A, Rinv, lane);
  store_mat<KB>(Rinv, ctl->W, lane);
  if (lane == 0) {
    ctl->done = 0;
    ctl->sweep = 1;
    ctl->polish = 0;
  }
}

}  // namespace meg
