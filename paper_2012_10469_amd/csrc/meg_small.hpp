// Small k x k FP64 solves run by one workgroup at the end of each sweep:
//   Rayleigh-Ritz on the current subspace (Section 3: eigenpairs of W^T M W),
//   the Cholesky-QR transform that orthonormalises the next block, and, at
//   the end of the inner solve, the exponentiation / normalisation of
//   Definition 1 and the cheap certificate with b_{r+1} (Section 3.1.1).
// All matrices live in LDS with row stride KB + 1 (bank-conflict padding).
#pragma once
#include "meg_device.hpp"

namespace meg {

// C = A^T B (all KB x KB, stride LD)
template <int KB, int NT>
__device__ void mm_tn(const double* A, const double* B, double* C) {
  constexpr int LD = KB + 1;
  for (int e = threadIdx.x; e < KB * KB; e += NT) {
    const int i = e / KB, j = e % KB;
    double s = 0.0;
#pragma unroll 8
    for (int l = 0; l < KB; ++l) s += A[l * LD + i] * B[l * LD + j];
    C[i * LD + j] = s;
  }
}

// C = A B
template <int KB, int NT>
__device__ void mm_nn(const double* A, const double* B, double* C) {
  constexpr int LD = KB + 1;
  for (int e = threadIdx.x; e < KB * KB; e += NT) {
    const int i = e / KB, j = e % KB;
    double s = 0.0;
#pragma unroll 8
    for (int l = 0; l < KB; ++l) s += A[i * LD + l] * B[l * LD + j];
    C[i * LD + j] = s;
  }
}

// Load a dense KB x KB (stride KB) global/LDS matrix into LDS stride LD.
template <int KB, int NT>
__device__ void load_mat(const double* src, double* dst) {
  constexpr int LD = KB + 1;
  for (int e = threadIdx.x; e < KB * KB; e += NT) dst[(e / KB) * LD + (e % KB)] = src[e];
}

template <int KB, int NT>
__device__ void store_mat(const double* src, double* dst) {
  constexpr int LD = KB + 1;
  for (int e = threadIdx.x; e < KB * KB; e += NT) dst[e] = src[(e / KB) * LD + (e % KB)];
}

// Cyclic parallel Jacobi (round-robin ordering) for symmetric A in LDS.
// On return A is (numerically) diagonal and A_in = S diag(A) S^T.
// `rot` needs 2 * KB doubles and 2 * KB ints worth of space (4 * KB doubles).
template <int KB, int NT>
__device__ void jacobi(double* A, double* S, double* rot) {
  constexpr int LD = KB + 1;
  constexpr int NP = KB / 2;
  __shared__ double s_norm[2];
  double* rc = rot;
  double* rs = rot + NP;
  int* rp = reinterpret_cast<int*>(rot + 2 * NP);
  int* rq = rp + NP;
  const int tid = threadIdx.x;
  for (int e = tid; e < KB * KB; e += NT) S[(e / KB) * LD + (e % KB)] = (e / KB == e % KB) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid < 64) {
      double off = 0.0, dia = 0.0;
      for (int e = tid; e < KB * KB; e += 64) {
        const double v = A[(e / KB) * LD + (e % KB)];
        if (e / KB == e % KB) dia += v * v; else off += v * v;
      }
      off = wave_sum(off);
      dia = wave_sum(dia);
      if (tid == 0) { s_norm[0] = off; s_norm[1] = dia; }
    }
    __syncthreads();
    if (!(s_norm[0] > 1e-30 * (s_norm[0] + s_norm[1]))) break;  // also exits on NaN
    for (int round = 0; round < KB - 1; ++round) {
      if (tid < NP) {
        // circle method: slot 0 fixed, slots 1..KB-1 rotate by `round`
        const int a = tid, b = KB - 1 - tid;
        const int pa = (a == 0) ? 0 : 1 + ((a - 1 + round) % (KB - 1));
        const int pb = 1 + ((b - 1 + round) % (KB - 1));
        const int p = min(pa, pb), q = max(pa, pb);
        const double apq = A[p * LD + q], app = A[p * LD + p], aqq = A[q * LD + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        rc[tid] = c; rs[tid] = s; rp[tid] = p; rq[tid] = q;
      }
      __syncthreads();
      for (int e = tid; e < NP * KB; e += NT) {  // rows: A <- J^T A
        const int mm = e / KB, j = e % KB;
        const int p = rp[mm], q = rq[mm];
        const double c = rc[mm], s = rs[mm];
        const double a = A[p * LD + j], b = A[q * LD + j];
        A[p * LD + j] = c * a - s * b;
        A[q * LD + j] = s * a + c * b;
      }
      __syncthreads();
      for (int e = tid; e < NP * KB; e += NT) {  // columns: A <- A J, S <- S J
        const int mm = e / KB, i = e % KB;
        const int p = rp[mm], q = rq[mm];
        const double c = rc[mm], s = rs[mm];
        double a = A[i * LD + p], b = A[i * LD + q];
        A[i * LD + p] = c * a - s * b;
        A[i * LD + q] = s * a + c * b;
        a = S[i * LD + p]; b = S[i * LD + q];
        S[i * LD + p] = c * a - s * b;
        S[i * LD + q] = s * a + c * b;
      }
      __syncthreads();
    }
  }
}

// Cholesky A = R^T R (R upper, written over A's upper triangle; lower zeroed),
// then Rinv = R^{-1} (upper).  Tiny pivots are floored to keep R invertible.
template <int KB, int NT>
__device__ void chol_inv(double* A, double* Rinv) {
  constexpr int LD = KB + 1;
  __shared__ double s_piv;
  const int tid = threadIdx.x;
  double scale = 0.0;
  for (int i = 0; i < KB; ++i) scale = fmax(scale, A[i * LD + i]);
  const double floor_piv = fmax(scale, 1e-300) * 1e-28;
  for (int j = 0; j < KB; ++j) {
    if (tid == 0) {
      double dj = A[j * LD + j];
      if (!(dj > floor_piv)) dj = floor_piv;
      s_piv = sqrt(dj);
      A[j * LD + j] = s_piv;
    }
    __syncthreads();
    const double rjj = s_piv;
    for (int c = j + 1 + tid; c < KB; c += NT) A[j * LD + c] /= rjj;
    __syncthreads();
    for (int e = tid; e < KB * KB; e += NT) {
      const int a = e / KB, b = e % KB;
      if (a > j && b >= a) A[a * LD + b] -= A[j * LD + a] * A[j * LD + b];
    }
    __syncthreads();
  }
  for (int e = tid; e < KB * KB; e += NT) {
    const int a = e / KB, b = e % KB;
    if (b < a) A[a * LD + b] = 0.0;
  }
  __syncthreads();
  // back substitution per column of the inverse: R X = I
  for (int c = tid; c < KB; c += NT) {
    for (int i = KB - 1; i >= 0; --i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int l = i + 1; l < KB; ++l) s -= A[i * LD + l] * Rinv[l * LD + c];
      Rinv[i * LD + c] = (i > c) ? 0.0 : s / A[i * LD + i];
    }
  }
  __syncthreads();
}

// Per-step operator coefficients: Yhat = V diag(ceff) V^T + opscale*Op + sdiag*I
// equals M_t - log(alpha) I + sigma I.  gmax is an upper bound of
// lambda_max(grad f(X_t)); by Weyl's inequality
//   lambda_min(V diag(c) V^T - eta G) >= min(0, min c) - eta gmax,
// so sigma = eta gmax - min(0, min c) (+ a small margin) makes Yhat >= 0 and
// subspace iteration targets the algebraically largest eigenvalues.  A tight
// gmax matters: the unwanted spectrum then starts near 0, which is what makes
// the (r+1)-th pair converge.  Single thread.
__device__ inline void setup_step(const Cfg& cfg, Ctl* ctl, double gmax) {
  const int r = cfg.r;
  double cmin = 0.0, cmax = 0.0;
  for (int l = 0; l < r; ++l) {
    cmin = fmin(cmin, ctl->c[l]);
    cmax = fmax(cmax, ctl->c[l]);
  }
  const double base = cfg.eta * gmax - cmin;
  const double sigma = base + 1e-3 * (fabs(base) + cmax) + 1e-30;
  ctl->gmax = gmax;
  ctl->sigma = sigma;
  if (cfg.kind == DENOISE_DENSE) {
    // G = X - M:  V c V^T - eta(alpha I + V d V^T - M) + sigma I
    for (int l = 0; l < KMAX; ++l) ctl->ceff[l] = (l < r) ? ctl->c[l] - cfg.eta * ctl->d[l] : 0.0;
    ctl->sdiag = sigma - cfg.eta * ctl->alpha;
    ctl->opscale = cfg.eta;
  } else {
    for (int l = 0; l < KMAX; ++l) ctl->ceff[l] = (l < r) ? ctl->c[l] : 0.0;
    ctl->sdiag = sigma;
    ctl->opscale = -cfg.eta;
  }
  ctl->info.t = ctl->t;
  ctl->info.sigma = sigma;
  ctl->info.f = ctl->fvalid ? ctl->f : __builtin_nan("");
}

// End of the inner solve: exponentiate and normalise (Definition 1), build
// the next factored iterate (alpha', d', c') and the certificate.
// theta[0..r] are the sorted Ritz values of Yhat.  Single thread.
__device__ inline void finish_step(const Cfg& cfg, Ctl* ctl, const double* theta, double* mu,
                                   double resid_max, int sweeps, int converged) {
  const int r = cfg.r;
  const double n = (double)cfg.n;
  const double la = log(ctl->alpha);
  for (int i = 0; i <= r; ++i) mu[i] = theta[i] + la - ctl->sigma;  // eigenvalues of M_t
  double m = mu[0];
  for (int i = 1; i <= r; ++i) m = fmax(m, mu[i]);
  double sr = 0.0;
  for (int i = 0; i < r; ++i) sr += exp(mu[i] - m);
  const double lse_r = m + log(sr);                        // log a_t
  const double lse_r1 = m + log(sr + exp(mu[r] - m));      // log b^{r+1}_t
  const double eps = eps_at(cfg, ctl->t);
  const double alpha_n = eps / (n - r);
  const double l1e = log1p(-eps);
  const double la_n = log(alpha_n);
  bool finite = isfinite(lse_r1);
  for (int l = 0; l < r; ++l) {
    const double lt = mu[l] - lse_r;        // log lambda~_l = mu_l - log a_t
    const double dl = (1.0 - eps) * exp(lt) - alpha_n;
    ctl->d[l] = dl;
    ctl->c[l] = l1e + lt - la_n;            // log((1-eps) lambda~_l) - log(alpha')
    finite = finite && isfinite(dl);
  }
  for (int l = r; l < KMAX; ++l) { ctl->d[l] = 0.0; ctl->c[l] = 0.0; }
  ctl->alpha = alpha_n;
  const double L = log(n - r) - log(eps) + mu[r] - lse_r1;
  Info& in = ctl->info;
  in.t = ctl->t;
  in.eps_t = eps;
  in.cert_L = L;
  in.cert_bound = fmax(2.0 * eps, L);
  in.cert_holds = (L <= 2.0 * eps) ? 1 : 0;
  in.inner_iters = sweeps;
  in.ritz_gap = mu[r - 1] - mu[r];
  in.resid_max = resid_max;
  in.resid_r1 = ctl->resid[r];
  in.mu_r1 = mu[r];
  in.sigma = ctl->sigma;
  in.converged = converged;
  if (!finite) ctl->status = 4;  // MEG_ERR_NUMERIC
  if (ctl->solve_tol > 0.0 && in.cert_bound <= ctl->solve_tol) ctl->stop = 1;
}

// One Rayleigh-Ritz / orthonormalisation step.  `sums` holds, stride KB:
//   C = Zin^T Zout, G = Zout^T Zout, P = V^T Zout (first r rows)
// where Zout = Yhat Q and Q = Zin W is orthonormal.  Run by all NT threads of
// the last workgroup.  `scr` needs 5 * KB * (KB + 1) + 8 * KB doubles.
template <int KB, int NT>
__device__ void small_sweep(const Cfg& cfg, Ctl* ctl, const double* sums, double* scr, int sweep,
                            int in_buf) {
  constexpr int LD = KB + 1;
  constexpr int MS = KB * LD;
  const int tid = threadIdx.x;
  double* A = scr;            // T, then diagonalised
  double* S = scr + MS;       // Ritz vectors (unsorted)
  double* B1 = scr + 2 * MS;  // W, then sorted S
  double* B2 = scr + 3 * MS;  // C, then G S, then Rinv
  double* B3 = scr + 4 * MS;  // G, then Ghat = S^T G S
  double* vec = scr + 5 * MS; // 8 * KB
  double* theta = vec;
  double* rho = vec + KB;
  double* rot = vec + 2 * KB;  // 4 * KB
  double* mu = vec + 6 * KB;   // KB + 1 <= 2 * KB
  __shared__ int s_perm[KMAX];
  __shared__ int s_final;
  __shared__ double s_rmax;

  load_mat<KB, NT>(ctl->W, B1);
  load_mat<KB, NT>(sums, B2);
  load_mat<KB, NT>(sums + KB * KB, B3);
  __syncthreads();
  mm_tn<KB, NT>(B1, B2, A);  // T = W^T C = Q^T Yhat Q
  __syncthreads();
  for (int e = tid; e < KB * KB; e += NT) {  // symmetrise
    const int i = e / KB, j = e % KB;
    if (i < j) {
      const double v = 0.5 * (A[i * LD + j] + A[j * LD + i]);
      A[i * LD + j] = v;
      A[j * LD + i] = v;
    }
  }
  __syncthreads();
  jacobi<KB, NT>(A, S, rot);
  if (tid == 0) {  // sort eigenvalues descending (selection sort, KB <= 32)
    uint32_t used = 0u;
    for (int i = 0; i < KB; ++i) {
      int best = -1;
      double bv = 0.0;
      for (int j = 0; j < KB; ++j) {
        const double v = A[j * LD + j];
        if (!((used >> j) & 1u) && (best < 0 || v > bv)) { best = j; bv = v; }
      }
      if (best < 0) best = i;  // NaN diagonal: keep position, flagged below
      used |= 1u << best;
      s_perm[i] = best;
      theta[i] = A[best * LD + best];
    }
  }
  __syncthreads();
  for (int e = tid; e < KB * KB; e += NT) {  // B1 <- sorted S
    const int i = e / KB, j = e % KB;
    B1[i * LD + j] = S[i * LD + s_perm[j]];
  }
  __syncthreads();
  mm_nn<KB, NT>(B3, B1, B2);  // G S
  __syncthreads();
  mm_tn<KB, NT>(B1, B2, B3);  // Ghat = S^T G S  (Gram of Zout S)
  __syncthreads();
  if (tid < KB) {  // Ritz residuals ||Yhat q s_i - theta_i q s_i||^2 = Ghat_ii - theta_i^2
    const double v = B3[tid * LD + tid] - theta[tid] * theta[tid];
    rho[tid] = sqrt(fmax(v, 0.0));
  }
  __syncthreads();
  if (tid == 0) {
    const int r = cfg.r;
    const double scale = fmax(fabs(theta[0]), 1e-300);
    // Residuals come from Ghat_ii - theta_i^2 in FP64: resolvable down to
    // ~sqrt(2^-53) of the scale; working-precision rounding sets another floor.
    const double floor_est = fmax(3e-8, 8.0 * cfg.unit_round) * scale;
    const double thr = fmax(cfg.inner_tol * scale, floor_est);
    double rmax = 0.0;
    bool finite = true;
    for (int i = 0; i < KB; ++i) finite = finite && isfinite(theta[i]) && isfinite(rho[i]);
    for (int i = 0; i < r; ++i) rmax = fmax(rmax, rho[i]);
    const bool cert_ok = !(cfg.cert_tol > 0.0) || rho[r] <= fmax(cfg.cert_tol, floor_est);
    int conv = (rmax <= thr && cert_ok) ? 1 : 0;
    // tolerance below the resolvable floor: two more sweeps once it is reached
    if (conv && cfg.inner_tol * scale < floor_est && ctl->polish < 2) {
      ctl->polish = ctl->polish + 1;
      conv = 0;
    }
    s_rmax = rmax;
    for (int i = 0; i < KB; ++i) { ctl->theta[i] = theta[i]; ctl->resid[i] = rho[i]; }
    int fin = ((conv && sweep >= cfg.min_inner) || sweep >= cfg.max_inner) ? 1 : 0;
    if (!finite) {
      ctl->status = 4;  // MEG_ERR_NUMERIC
      ctl->stop = 1;
      fin = 1;
    } else if (fin) {
      finish_step(cfg, ctl, theta, mu, rmax, sweep, conv);
    }
    s_final = fin;
  }
  __syncthreads();
  if (s_final) {
    // Ritz vectors of span(Q): Q S = Zin (W S)
    double* W = B2;
    load_mat<KB, NT>(ctl->W, W);
    __syncthreads();
    mm_nn<KB, NT>(W, B1, A);
    __syncthreads();
    store_mat<KB, NT>(A, ctl->Wfin);
    if (tid == 0) {
      ctl->src = in_buf;
      ctl->done = 1;
    }
    return;
  }
  // Next basis Q' = Zout S R^{-1} with Ghat = R^T R (Cholesky QR, FP64)
  chol_inv<KB, NT>(B3, B2);
  mm_nn<KB, NT>(B1, B2, A);  // W' = S R^{-1}
  __syncthreads();
  store_mat<KB, NT>(A, ctl->W);
  for (int e = tid; e < KB * KB; e += NT) ctl->Pin[e] = sums[2 * KB * KB + e];  // V^T Zout
  if (tid == 0) ctl->sweep = sweep + 1;
}

// Orthonormalising transform of a fresh basis Qw with Gram H = Qw^T Qw:
// W = R^{-1} (H = R^T R), Pin = V^T Qw = H[0:r, :].  All threads.
template <int KB, int NT>
__device__ void basis_setup(const Cfg& cfg, Ctl* ctl, const double* gram, double* scr) {
  constexpr int LD = KB + 1;
  constexpr int MS = KB * LD;
  double* A = scr;
  double* Rinv = scr + MS;
  for (int e = threadIdx.x; e < KB * KB; e += NT) ctl->Pin[e] = gram[e];
  load_mat<KB, NT>(gram, A);
  __syncthreads();
  chol_inv<KB, NT>(A, Rinv);
  store_mat<KB, NT>(Rinv, ctl->W);
  if (threadIdx.x == 0) {
    ctl->done = 0;
    ctl->sweep = 1;
    ctl->polish = 0;
  }
}

}  // namespace meg
