// Host runtime of the low-rank MEG library: the C ABI declared in include/meg.h.
//
// One context = one problem instance on one device stream.  The runtime
// validates arguments, allocates the device state, builds the first iterate of
// Algorithm 2 and enqueues the per-step kernels (meg_kernels.hpp).  A step is
// captured once into a HIP graph (gradient/prep, max_inner sweeps, finalize)
// and replayed; kernels of sweeps after convergence exit at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/meg.h"
#include "meg_kernels.hpp"

using namespace meg;

namespace {

constexpr uint32_t kStateMagic = 0x4d454731u;  // "MEG1"
constexpr int kApplyNT = 256;
constexpr int kCsrRows = 8;
constexpr int kFinNT = 256;
constexpr int kFinRows = 16;


Red make_red(const meg_ctx_s* c, int nwg, int plen);

}  // namespace

struct meg_ctx_s {
  Cfg cfg{};
  meg_params params{};
  meg_objective obj{};
  hipStream_t stream = nullptr;
  size_t esize = 0;  // sizeof(T)
  void* Qw = nullptr;
  void* Za = nullptr;
  void* Zb = nullptr;
  void* g = nullptr;
  Ctl* ctl = nullptr;
  double* part = nullptr;
  double* gpart = nullptr;
  unsigned* cnt = nullptr;
  size_t part_elems = 0, gpart_elems = 0, cnt_elems = 0;
  Ctl* h_ctl = nullptr;  // pinned host mirror
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool use_graph = false;
  bool failed = false;
};

namespace {

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

Red make_red(const meg_ctx_s* c, int nwg, int plen) {
  Red r;
  r.part = c->part;
  r.gpart = c->gpart;
  r.cnt = c->cnt;
  r.nwg = nwg;
  r.gsz = std::max(1, (int)std::ceil(std::sqrt((double)nwg)));
  r.ngroups = ceil_div(nwg, r.gsz);
  r.plen = plen;
  return r;
}

void red_need(int nwg, int plen, size_t& part, size_t& gpart, size_t& cnt) {
  const int gsz = std::max(1, (int)std::ceil(std::sqrt((double)nwg)));
  const int ng = ceil_div(nwg, gsz);
  part = std::max(part, (size_t)nwg * plen);
  gpart = std::max(gpart, (size_t)ng * plen);
  cnt = std::max(cnt, (size_t)ng + 1);
}

int dense_rpw(int kb, size_t es) {
  const size_t bytes = (size_t)kb * es;
  return bytes <= 64 ? 4 : (bytes <= 128 ? 2 : 1);
}

// ---- small host PRNG (SplitMix64 + Box-Muller) for the extra start columns
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// Host basis: columns 0..q-1 = V (n x q col-major), q..k-1 = seeded Gaussian
// columns orthonormalised against all previous ones (two passes of modified
// Gram-Schmidt in FP64).  Output row-major n x k.
bool build_basis(int64_t n, int k, int q, const double* V, uint64_t seed, std::vector<double>& out) {
  std::vector<double> B((size_t)n * k);
  for (int j = 0; j < q; ++j)
    for (int64_t i = 0; i < n; ++i) B[(size_t)j * n + i] = V[(size_t)j * n + i];
  SplitMix rng{seed * 0x2545f4914f6cdd1dull + 12345};
  for (int j = q; j < k; ++j) {
    double* b = &B[(size_t)j * n];
    for (int attempt = 0; attempt < 4; ++attempt) {
      for (int64_t i = 0; i < n; ++i) b[i] = rng.normal();
      for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < j; ++l) {
          const double* a = &B[(size_t)l * n];
          double s = 0;
          for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
          for (int64_t i = 0; i < n; ++i) b[i] -= s * a[i];
        }
      double nr = 0;
      for (int64_t i = 0; i < n; ++i) nr += b[i] * b[i];
      nr = std::sqrt(nr);
      if (nr > 1e-8) {
        for (int64_t i = 0; i < n; ++i) b[i] /= nr;
        break;
      }
      if (attempt == 3) return false;
    }
  }
  out.assign((size_t)n * k, 0.0);
  for (int j = 0; j < k; ++j)
    for (int64_t i = 0; i < n; ++i) out[(size_t)i * k + j] = B[(size_t)j * n + i];
  return true;
}

meg_status hip_fail(meg_ctx c) {
  if (c) c->failed = true;
  return MEG_ERR_DEVICE;
}

#define HIPCHK(ctx, x)                               \
  do {                                               \
    if ((x) != hipSuccess) return hip_fail(ctx);     \
  } while (0)

// ---------------------------------------------------------------------------
// kernel launch helpers, dispatched on T (element type) and KB (block size)
// ---------------------------------------------------------------------------
template <typename T, int KB>
struct Launch {
  static void* zbuf(meg_ctx c, int i) { return i == 0 ? c->Qw : (i == 1 ? c->Za : c->Zb); }

  static void sizes(const Cfg& cfg, size_t& part, size_t& gpart, size_t& cnt) {
    const int64_t n = cfg.n;
    red_need(ceil_div(n, 4), 2, part, gpart, cnt);                    // grad / objective
    red_need(ceil_div(n, kCsrRows), 3 * KB * KB, part, gpart, cnt);   // csr apply
    const int rows = dense_rpw(KB, sizeof(T)) * (kApplyNT / 64);
    red_need(ceil_div(n, rows), 3 * KB * KB, part, gpart, cnt);       // dense apply
    red_need(ceil_div(n, kFinRows), KB * KB, part, gpart, cnt);       // finalize
    red_need(1024, 2, part, gpart, cnt);                              // sumsq
  }

  static void prep(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    if (cfg.kind == MASKED_CSR) {
      const int nwg = ceil_div(cfg.n, 4);
      hipLaunchKernelGGL((k_grad_masked<T, KB>), dim3(nwg), dim3(256), 0, c->stream, cfg, c->ctl,
                         c->obj.row_ptr, c->obj.col, (const T*)c->obj.val, (const T*)c->Qw, (T*)c->g,
                         make_red(c, nwg, 2));
    } else {
      hipLaunchKernelGGL(k_prep, dim3(1), dim3(64), 0, c->stream, cfg, c->ctl);
    }
  }

  static void sweep(meg_ctx c, int s) {
    const Cfg& cfg = c->cfg;
    const int in = (s == 1) ? 0 : ((s % 2 == 0) ? 1 : 2);
    const int out = (s == 1) ? 1 : ((s % 2 == 0) ? 2 : 1);
    const T* Zin = (const T*)zbuf(c, in);
    T* Zout = (T*)zbuf(c, out);
    if (cfg.kind == MASKED_CSR || cfg.kind == LINEAR_CSR) {
      const int nwg = ceil_div(cfg.n, kCsrRows);
      const T* gv = (cfg.kind == MASKED_CSR) ? (const T*)c->g : (const T*)c->obj.val;
      hipLaunchKernelGGL((k_apply_csr<T, KB, kCsrRows, kApplyNT>), dim3(nwg), dim3(kApplyNT), 0, c->stream, cfg,
                         c->ctl, c->obj.row_ptr, c->obj.col, gv, (const T*)c->Qw, Zin, Zout,
                         make_red(c, nwg, 3 * KB * KB), s, in);
    } else {
      const int rpw = dense_rpw(KB, sizeof(T));
      const int rows = rpw * (kApplyNT / 64);
      const int nwg = ceil_div(cfg.n, rows);
      const Red red = make_red(c, nwg, 3 * KB * KB);
      const T* D = (const T*)c->obj.dense;
      if (rpw == 4)
        hipLaunchKernelGGL((k_apply_dense<T, KB, 4, kApplyNT>), dim3(nwg), dim3(kApplyNT), 0, c->stream, cfg,
                           c->ctl, D, (const T*)c->Qw, Zin, Zout, red, s, in);
      else if (rpw == 2)
        hipLaunchKernelGGL((k_apply_dense<T, KB, 2, kApplyNT>), dim3(nwg), dim3(kApplyNT), 0, c->stream, cfg,
                           c->ctl, D, (const T*)c->Qw, Zin, Zout, red, s, in);
      else
        hipLaunchKernelGGL((k_apply_dense<T, KB, 1, kApplyNT>), dim3(nwg), dim3(kApplyNT), 0, c->stream, cfg,
                           c->ctl, D, (const T*)c->Qw, Zin, Zout, red, s, in);
    }
  }

  static void finalize(meg_ctx c, int mode) {
    const int nwg = ceil_div(c->cfg.n, kFinRows);
    hipLaunchKernelGGL((k_finalize<T, KB, kFinRows, kFinNT>), dim3(nwg), dim3(kFinNT), 0, c->stream, c->cfg,
                       c->ctl, (T*)c->Qw, (const T*)c->Za, (const T*)c->Zb, make_red(c, nwg, KB * KB), mode);
  }

  static void objective(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    const int nwg = ceil_div(cfg.n, 4);
    if (cfg.kind == LINEAR_DENSE || cfg.kind == DENOISE_DENSE)
      hipLaunchKernelGGL((k_objective_dense<T, KB>), dim3(nwg), dim3(256), 0, c->stream, cfg, c->ctl,
                         (const T*)c->obj.dense, (const T*)c->Qw, make_red(c, nwg, 2));
    else
      hipLaunchKernelGGL((k_objective_csr<T, KB>), dim3(nwg), dim3(256), 0, c->stream, cfg, c->ctl,
                         c->obj.row_ptr, c->obj.col, (const T*)c->obj.val, (const T*)c->Qw,
                         make_red(c, nwg, 2));
  }

  static void data_norm(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    int64_t rows, cols, ld;
    const T* x;
    if (cfg.kind == LINEAR_DENSE || cfg.kind == DENOISE_DENSE) {
      rows = cfg.n; cols = cfg.n; ld = cfg.ld; x = (const T*)c->obj.dense;
    } else {
      rows = 1; cols = std::max<int64_t>(cfg.nnz, 1); ld = 0; x = (const T*)c->obj.val;
      if (cfg.nnz == 0) { rows = 0; }
    }
    const int64_t total = rows * cols;
    const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (total + 255) / 256));
    hipLaunchKernelGGL((k_sumsq<T>), dim3(nwg), dim3(256), 0, c->stream, x, rows, cols, ld, c->ctl,
                       make_red(c, nwg, 2));
  }

  static void step(meg_ctx c) {
    prep(c);
    for (int s = 1; s <= c->cfg.max_inner; ++s) sweep(c, s);
    finalize(c, 0);
  }
};

template <typename T, int KB>
struct DoProfile {
  static void run(meg_ctx c, hipEvent_t* ev) {
    hipEventRecord(ev[0], c->stream);
    Launch<T, KB>::prep(c);
    hipEventRecord(ev[1], c->stream);
    for (int s = 1; s <= c->cfg.max_inner; ++s) {
      Launch<T, KB>::sweep(c, s);
      hipEventRecord(ev[1 + s], c->stream);
    }
    Launch<T, KB>::finalize(c, 0);
    hipEventRecord(ev[2 + c->cfg.max_inner], c->stream);
  }
};

template <template <typename, int> class F, typename... Args>
void dispatch(meg_ctx c, Args&&... args) {
  const bool dbl = c->esize == 8;
  if (c->cfg.k == 16) {
    if (dbl) F<double, 16>::run(c, args...); else F<float, 16>::run(c, args...);
  } else {
    if (dbl) F<double, 32>::run(c, args...); else F<float, 32>::run(c, args...);
  }
}

template <typename T, int KB> struct DoStep { static void run(meg_ctx c) { Launch<T, KB>::step(c); } };
template <typename T, int KB> struct DoFinalize { static void run(meg_ctx c, int m) { Launch<T, KB>::finalize(c, m); } };
template <typename T, int KB> struct DoObjective { static void run(meg_ctx c) { Launch<T, KB>::objective(c); } };
template <typename T, int KB> struct DoNorm { static void run(meg_ctx c) { Launch<T, KB>::data_norm(c); } };
template <typename T, int KB> struct DoSizes {
  static void run(meg_ctx c, size_t* p, size_t* g, size_t* n) { Launch<T, KB>::sizes(c->cfg, *p, *g, *n); }
};

// Eigenvalues/vectors of a small symmetric matrix (host, cyclic Jacobi, FP64).
// A is m x m row-major (destroyed); w gets eigenvalues, S (m x m) eigenvectors
// as columns.
void host_sym_eig(std::vector<double>& A, int m, std::vector<double>& w, std::vector<double>& S) {
  S.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) S[(size_t)i * m + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        const double v = A[(size_t)i * m + j] * A[(size_t)i * m + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[(size_t)p * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double tau = (A[(size_t)q * m + q] - A[(size_t)p * m + p]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        for (int k = 0; k < m; ++k) {  // rows
          const double a = A[(size_t)p * m + k], b = A[(size_t)q * m + k];
          A[(size_t)p * m + k] = cs * a - sn * b;
          A[(size_t)q * m + k] = sn * a + cs * b;
        }
        for (int k = 0; k < m; ++k) {  // columns
          double a = A[(size_t)k * m + p], b = A[(size_t)k * m + q];
          A[(size_t)k * m + p] = cs * a - sn * b;
          A[(size_t)k * m + q] = sn * a + cs * b;
          a = S[(size_t)k * m + p];
          b = S[(size_t)k * m + q];
          S[(size_t)k * m + p] = cs * a - sn * b;
          S[(size_t)k * m + q] = sn * a + cs * b;
        }
      }
  }
  w.resize(m);
  for (int i = 0; i < m; ++i) w[i] = A[(size_t)i * m + i];
}

// Lanczos (full reorthogonalisation, host recurrence, device matvec) for the
// extreme eigenvalues of the data operator: C (linear), M (denoising) or the
// masked values P_Omega(M).  Returns bounds widened by the Ritz residuals.
template <typename T>
meg_status lanczos_extremes(meg_ctx c, double* lmin, double* lmax) {
  const Cfg& cfg = c->cfg;
  const int64_t n = cfg.n;
  const int m = (int)std::min<int64_t>(n, 48);
  T* dx = nullptr;
  double* dy = nullptr;
  if (hipMalloc((void**)&dx, n * sizeof(T)) != hipSuccess) return MEG_ERR_OUT_OF_MEMORY;
  if (hipMalloc((void**)&dy, n * sizeof(double)) != hipSuccess) {
    (void)hipFree(dx);
    return MEG_ERR_OUT_OF_MEMORY;
  }
  std::vector<double> Vs((size_t)(m + 1) * n), y(n), w(n);
  std::vector<T> xt(n);
  std::vector<double> al(m, 0.0), be(m, 0.0);
  SplitMix rng{c->params.seed ^ 0x6c616e637a6f73ull};
  double nrm = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    Vs[i] = rng.normal();
    nrm += Vs[i] * Vs[i];
  }
  nrm = std::sqrt(nrm);
  for (int64_t i = 0; i < n; ++i) Vs[i] /= nrm;
  int meff = m;
  meg_status st = MEG_OK;
  for (int j = 0; j < m; ++j) {
    const double* v = &Vs[(size_t)j * n];
    for (int64_t i = 0; i < n; ++i) xt[i] = (T)v[i];
    if (hipMemcpy(dx, xt.data(), n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) { st = hip_fail(c); break; }
    hipLaunchKernelGGL((k_matvec<T>), dim3(ceil_div(n, 4)), dim3(256), 0, c->stream, cfg, (const T*)c->obj.dense,
                       c->obj.row_ptr, c->obj.col, (const T*)c->obj.val, (const T*)dx, dy);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(y.data(), dy, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
      st = hip_fail(c);
      break;
    }
    double a = 0.0;
    for (int64_t i = 0; i < n; ++i) a += y[i] * v[i];
    for (int64_t i = 0; i < n; ++i) w[i] = y[i] - a * v[i] - (j > 0 ? be[j - 1] * Vs[(size_t)(j - 1) * n + i] : 0.0);
    for (int pass = 0; pass < 2; ++pass)
      for (int l = 0; l <= j; ++l) {
        const double* u = &Vs[(size_t)l * n];
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += u[i] * w[i];
        for (int64_t i = 0; i < n; ++i) w[i] -= s * u[i];
      }
    double b = 0.0;
    for (int64_t i = 0; i < n; ++i) b += w[i] * w[i];
    b = std::sqrt(b);
    al[j] = a;
    be[j] = b;
    if (!(b > 1e-10 * (std::fabs(a) + 1e-300))) {
      meff = j + 1;
      be[j] = 0.0;
      break;
    }
    double* vn = &Vs[(size_t)(j + 1) * n];
    for (int64_t i = 0; i < n; ++i) vn[i] = w[i] / b;
  }
  (void)hipFree(dx);
  (void)hipFree(dy);
  if (st != MEG_OK) return st;
  std::vector<double> Tm((size_t)meff * meff, 0.0), ev, S;
  for (int j = 0; j < meff; ++j) {
    Tm[(size_t)j * meff + j] = al[j];
    if (j + 1 < meff) Tm[(size_t)j * meff + j + 1] = Tm[(size_t)(j + 1) * meff + j] = be[j];
  }
  host_sym_eig(Tm, meff, ev, S);
  int imin = 0, imax = 0;
  for (int i = 1; i < meff; ++i) {
    if (ev[i] < ev[imin]) imin = i;
    if (ev[i] > ev[imax]) imax = i;
  }
  const double bl = be[meff - 1];
  const double rmin = std::fabs(bl * S[(size_t)(meff - 1) * meff + imin]);
  const double rmax = std::fabs(bl * S[(size_t)(meff - 1) * meff + imax]);
  const double spread = ev[imax] - ev[imin];
  *lmin = ev[imin] - rmin - 1e-6 * spread;
  *lmax = ev[imax] + rmax + 1e-6 * spread;
  return MEG_OK;
}

meg_status copy_ctl_to_host(meg_ctx c) {
  HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MEG_OK;
}

void fill_info(const Ctl& h, meg_step_info* o) {
  const Info& in = h.info;
  o->t = in.t;
  o->f = in.f;
  o->eps_t = in.eps_t;
  o->cert_L = in.cert_L;
  o->cert_bound = in.cert_bound;
  o->cert_holds = in.cert_holds;
  o->inner_iters = in.inner_iters;
  o->ritz_gap = in.ritz_gap;
  o->resid_max = in.resid_max;
  o->mu_r1 = in.mu_r1;
  o->sigma = in.sigma;
  o->converged = in.converged;
  o->reserved = 0;
  o->resid_r1 = in.resid_r1;
}

// Write host iterate (V n x q col-major, d, alpha, t) + fresh basis into the device.
meg_status upload_iterate(meg_ctx c, const double* V, int q, const double* d, double alpha, int64_t t) {
  const Cfg& cfg = c->cfg;
  std::vector<double> B;
  if (!build_basis(cfg.n, cfg.k, q, V, c->params.seed + (uint64_t)t * 7919u, B)) return MEG_ERR_INVALID_ARG;
  const size_t cnt = (size_t)cfg.n * cfg.k;
  if (c->esize == 8) {
    HIPCHK(c, hipMemcpyAsync(c->Qw, B.data(), cnt * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::vector<float> Bf(cnt);
    for (size_t i = 0; i < cnt; ++i) Bf[i] = (float)B[i];
    HIPCHK(c, hipMemcpyAsync(c->Qw, Bf.data(), cnt * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  Ctl& h = *c->h_ctl;
  h.alpha = alpha;
  for (int l = 0; l < KMAX; ++l) {
    const double dl = (l < q) ? d[l] : 0.0;
    h.d[l] = (l < cfg.r) ? dl : 0.0;
    h.c[l] = (l < cfg.r) ? std::log(alpha + h.d[l]) - std::log(alpha) : 0.0;
  }
  h.t = t;
  h.done = 0;
  h.sweep = 1;
  h.src = 0;
  h.stop = 0;
  h.status = 0;
  h.fvalid = 0;
  h.solve_tol = 0.0;
  std::memset(&h.info, 0, sizeof(Info));
  h.info.t = t - 1;
  HIPCHK(c, hipMemcpyAsync(c->ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  dispatch<DoFinalize>(c, 1);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MEG_OK;
}

meg_status build_graph(meg_ctx c) {
  if (!c->use_graph) return MEG_OK;
  if (c->gexec) return MEG_OK;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  dispatch<DoStep>(c);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(c->stream, &g) != hipSuccess || !g) return hip_fail(c);
  c->graph = g;
  if (hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) != hipSuccess) return hip_fail(c);
  return MEG_OK;
}

meg_status enqueue_step(meg_ctx c) {
  if (c->use_graph) {
    meg_status s = build_graph(c);
    if (s != MEG_OK) return s;
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  } else {
    dispatch<DoStep>(c);
    HIPCHK(c, hipGetLastError());
  }
  return MEG_OK;
}

meg_status check_ctx(meg_ctx c) {
  if (!c) return MEG_ERR_INVALID_ARG;
  if (c->failed) return MEG_ERR_STATE;
  return MEG_OK;
}

meg_status validate(const meg_params* p, const meg_objective* o, const meg_start* s, int* kout) {
  if (!p || !o || !s) return MEG_ERR_INVALID_ARG;
  if (p->n < 2 || p->r < 1 || p->r > p->n - 1) return MEG_ERR_INVALID_ARG;
  if (p->oversample < 0) return MEG_ERR_INVALID_ARG;
  const int k = meg_block_size(p->r, p->oversample);
  if (k == 0 || k > p->n) return MEG_ERR_INVALID_ARG;
  if (p->prec < MEG_PREC_F64 || p->prec > MEG_PREC_F32_BF16X3) return MEG_ERR_INVALID_ARG;
  if (!(p->eta > 0.0) || !std::isfinite(p->eta)) return MEG_ERR_INVALID_ARG;
  if (!(p->eps_scale > 0.0) || !std::isfinite(p->eps_c) || !(p->eps_pow >= 0.0)) return MEG_ERR_INVALID_ARG;
  if (p->eps_c + 1.0 <= 0.0) return MEG_ERR_INVALID_ARG;
  const double eps0 = p->eps_scale / std::pow(p->eps_c + 1.0, p->eps_pow);
  if (!(eps0 > 0.0 && eps0 <= 0.75)) return MEG_ERR_INVALID_ARG;
  if (p->min_inner < 1 || p->max_inner < p->min_inner || p->max_inner > 64) return MEG_ERR_INVALID_ARG;
  if (!(p->inner_tol >= 0.0) || !(p->cert_tol >= 0.0)) return MEG_ERR_INVALID_ARG;
  switch (o->kind) {
    case MEG_GRAD_LINEAR_DENSE:
    case MEG_GRAD_DENOISE_DENSE:
      if (!o->dense || o->ld < p->n) return MEG_ERR_INVALID_ARG;
      if (p->prec == MEG_PREC_F32_BF16X3) return MEG_ERR_UNSUPPORTED;
      break;
    case MEG_GRAD_LINEAR_CSR:
    case MEG_GRAD_MASKED_CSR:
      if (!o->row_ptr || o->nnz < 0 || (o->nnz > 0 && (!o->col || !o->val))) return MEG_ERR_INVALID_ARG;
      if (o->nnz > 2147483647LL) return MEG_ERR_INVALID_ARG;
      if (p->prec == MEG_PREC_F32_BF16X3) return MEG_ERR_UNSUPPORTED;
      break;
    case MEG_GRAD_QUADMEAS:
      return MEG_ERR_UNSUPPORTED;
    default:
      return MEG_ERR_INVALID_ARG;
  }
  if (s->q < 1 || s->q > p->r || !s->V0 || !s->lambda0) return MEG_ERR_INVALID_ARG;
  double sum = 0.0;
  for (int i = 0; i < s->q; ++i) {
    if (!(s->lambda0[i] >= 0.0)) return MEG_ERR_INVALID_ARG;
    sum += s->lambda0[i];
  }
  if (std::fabs(sum - 1.0) > 1e-8) return MEG_ERR_INVALID_ARG;
  // orthonormal start columns
  for (int a = 0; a < s->q; ++a)
    for (int b = a; b < s->q; ++b) {
      double dot = 0.0;
      for (int64_t i = 0; i < p->n; ++i) dot += s->V0[(size_t)a * p->n + i] * s->V0[(size_t)b * p->n + i];
      if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-6) return MEG_ERR_INVALID_ARG;
    }
  *kout = k;
  return MEG_OK;
}

void free_ctx(meg_ctx c) {
  if (!c) return;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  void* bufs[] = {c->Qw, c->Za, c->Zb, c->g, c->ctl, c->part, c->gpart, c->cnt};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  delete c;
}

}  // namespace

extern "C" {

int32_t meg_block_size(int32_t r, int32_t oversample) {
  if (r < 1 || oversample < 0) return 0;
  const int need = r + 1 + oversample;
  const int k = ((need + 15) / 16) * 16;
  return k <= KMAX ? k : 0;
}

const char* meg_status_str(meg_status s) {
  switch (s) {
    case MEG_OK: return "ok";
    case MEG_ERR_INVALID_ARG: return "invalid argument";
    case MEG_ERR_OUT_OF_MEMORY: return "out of device memory";
    case MEG_ERR_DEVICE: return "device (HIP) error";
    case MEG_ERR_NUMERIC: return "non-finite value in the solver";
    case MEG_ERR_NOT_CONVERGED: return "inner solver did not converge";
    case MEG_ERR_STATE: return "context failed earlier or bad state";
    case MEG_ERR_UNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

meg_status meg_init(meg_ctx* out, const meg_params* params, const meg_objective* obj, const meg_start* start,
                    void* stream) {
  if (!out) return MEG_ERR_INVALID_ARG;
  *out = nullptr;
  int k = 0;
  meg_status st = validate(params, obj, start, &k);
  if (st != MEG_OK) return st;
  meg_ctx c = new (std::nothrow) meg_ctx_s();
  if (!c) return MEG_ERR_OUT_OF_MEMORY;
  c->params = *params;
  c->obj = *obj;
  c->stream = (hipStream_t)stream;
  c->esize = (params->prec == MEG_PREC_F64) ? 8 : 4;
  Cfg& cfg = c->cfg;
  cfg.n = params->n;
  cfg.ld = obj->ld;
  cfg.nnz = obj->nnz;
  cfg.lda = obj->lda;
  cfg.m = obj->m;
  cfg.batch_steps = obj->batch_steps;
  cfg.r = params->r;
  cfg.k = k;
  cfg.kind = obj->kind;
  cfg.prec = params->prec;
  cfg.min_inner = params->min_inner;
  cfg.max_inner = params->max_inner;
  cfg.batch = obj->batch;
  cfg.eta = params->eta;
  cfg.eps_scale = params->eps_scale;
  cfg.eps_c = params->eps_c;
  cfg.eps_pow = params->eps_pow;
  cfg.inner_tol = params->inner_tol > 0 ? params->inner_tol : (c->esize == 8 ? 1e-10 : 1e-6);
  cfg.unit_round = (c->esize == 8) ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
  cfg.cert_tol = params->cert_tol;
  c->use_graph = !(params->flags & MEG_FLAG_NO_GRAPH) && stream != nullptr;

  size_t pe = 0, ge = 0, ce = 0;
  dispatch<DoSizes>(c, &pe, &ge, &ce);
  const size_t zbytes = (size_t)cfg.n * k * c->esize;
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 256)) == hipSuccess; };
  bool ok = alloc(&c->Qw, zbytes) && alloc(&c->Za, zbytes) && alloc(&c->Zb, zbytes) &&
            alloc((void**)&c->ctl, sizeof(Ctl)) && alloc((void**)&c->part, pe * 8) &&
            alloc((void**)&c->gpart, ge * 8) && alloc((void**)&c->cnt, ce * sizeof(unsigned));
  if (ok && obj->kind == MEG_GRAD_MASKED_CSR) ok = alloc(&c->g, (size_t)std::max<int64_t>(obj->nnz, 1) * c->esize);
  if (ok) ok = hipHostMalloc((void**)&c->h_ctl, sizeof(Ctl)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_ctx(c);
    return MEG_ERR_OUT_OF_MEMORY;
  }
  c->part_elems = pe;
  c->gpart_elems = ge;
  c->cnt_elems = ce;
  if (hipMemsetAsync(c->cnt, 0, ce * sizeof(unsigned), c->stream) != hipSuccess ||
      hipMemsetAsync(c->ctl, 0, sizeof(Ctl), c->stream) != hipSuccess) {
    free_ctx(c);
    return MEG_ERR_DEVICE;
  }
  // CSR structure check before any kernel reads through the indices
  if (obj->kind == MEG_GRAD_LINEAR_CSR || obj->kind == MEG_GRAD_MASKED_CSR) {
    int h_err = 0;
    int* d_err = (int*)c->cnt;  // zeroed above; reset below
    hipLaunchKernelGGL(k_check_csr, dim3((unsigned)std::min<int64_t>(1024, (cfg.n + 255) / 256)), dim3(256), 0,
                       c->stream, obj->row_ptr, obj->col, cfg.n, cfg.nnz, d_err);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemset(c->cnt, 0, ce * sizeof(unsigned)) != hipSuccess) {
      free_ctx(c);
      return MEG_ERR_DEVICE;
    }
    if (h_err) {
      free_ctx(c);
      return MEG_ERR_INVALID_ARG;
    }
  }
  // data norm (sets ctl->data_norm)
  dispatch<DoNorm>(c);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    free_ctx(c);
    return MEG_ERR_DEVICE;
  }
  // extreme eigenvalues of the data operator (shift of the subspace iteration)
  {
    double lmin = 0.0, lmax = 0.0;
    st = (c->esize == 8) ? lanczos_extremes<double>(c, &lmin, &lmax) : lanczos_extremes<float>(c, &lmin, &lmax);
    if (st == MEG_OK) st = copy_ctl_to_host(c);
    if (st != MEG_OK) {
      free_ctx(c);
      return st;
    }
    c->h_ctl->op_lmin = lmin;
    c->h_ctl->op_lmax = lmax;
    if (hipMemcpy(c->ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice) != hipSuccess) {
      free_ctx(c);
      return MEG_ERR_DEVICE;
    }
  }
  // X_1 = (1 - eps_0) X_0 + (eps_0 / n) I: alpha = eps_0/n, d = (1 - eps_0) lambda_0
  const double eps0 = cfg.eps_scale / std::pow(cfg.eps_c + 1.0, cfg.eps_pow);
  std::vector<double> d(start->q);
  for (int i = 0; i < start->q; ++i) d[i] = (1.0 - eps0) * start->lambda0[i];
  st = upload_iterate(c, start->V0, start->q, d.data(), eps0 / (double)cfg.n, 1);
  if (st != MEG_OK) {
    free_ctx(c);
    return st;
  }
  *out = c;
  return MEG_OK;
}

meg_status meg_step(meg_ctx c, meg_step_info* info) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (info) {
    dispatch<DoObjective>(c);
    HIPCHK(c, hipGetLastError());
  }
  st = enqueue_step(c);
  if (st != MEG_OK) return st;
  if (!info) return MEG_OK;
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  fill_info(*c->h_ctl, info);
  if (c->h_ctl->status) return (meg_status)c->h_ctl->status;
  if ((c->params.flags & MEG_FLAG_STRICT) && !info->converged) return MEG_ERR_NOT_CONVERGED;
  return MEG_OK;
}

meg_status meg_solve(meg_ctx c, int64_t max_iters, double tol, meg_step_info* last) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (max_iters < 0) return MEG_ERR_INVALID_ARG;
  // arm the device-side stop rule
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  c->h_ctl->solve_tol = tol > 0 ? tol : 0.0;
  c->h_ctl->stop = 0;
  HIPCHK(c, hipMemcpyAsync(&c->ctl->solve_tol, &c->h_ctl->solve_tol, sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(&c->ctl->stop, &c->h_ctl->stop, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  const int64_t chunk = 16;
  int64_t done = 0;
  while (done < max_iters) {
    const int64_t m = std::min<int64_t>(chunk, max_iters - done);
    for (int64_t i = 0; i < m; ++i) {
      st = enqueue_step(c);
      if (st != MEG_OK) return st;
    }
    done += m;
    if (tol > 0 || done >= max_iters) {
      st = copy_ctl_to_host(c);
      if (st != MEG_OK) return st;
      if (c->h_ctl->stop || c->h_ctl->status) break;
    }
  }
  if (done == 0) {
    st = copy_ctl_to_host(c);
    if (st != MEG_OK) return st;
  }
  const int32_t status = c->h_ctl->status;
  if (last) {
    fill_info(*c->h_ctl, last);
    last->f = __builtin_nan("");
  }
  // disarm
  c->h_ctl->solve_tol = 0.0;
  c->h_ctl->stop = 0;
  HIPCHK(c, hipMemcpyAsync(&c->ctl->solve_tol, &c->h_ctl->solve_tol, sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(&c->ctl->stop, &c->h_ctl->stop, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return status ? (meg_status)status : MEG_OK;
}

meg_status meg_certificate(meg_ctx c, meg_step_info* out) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!out) return MEG_ERR_INVALID_ARG;
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  fill_info(*c->h_ctl, out);
  return MEG_OK;
}

meg_status meg_objective_value(meg_ctx c, double* f) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!f) return MEG_ERR_INVALID_ARG;
  dispatch<DoObjective>(c);
  HIPCHK(c, hipGetLastError());
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  *f = c->h_ctl->f;
  return MEG_OK;
}

meg_status meg_get_iterate(meg_ctx c, double* V, double* d, double* alpha, int64_t* t) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  const Cfg& cfg = c->cfg;
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  if (V) {
    const size_t cnt = (size_t)cfg.n * cfg.k;
    std::vector<double> B(cnt);
    if (c->esize == 8) {
      HIPCHK(c, hipMemcpy(B.data(), c->Qw, cnt * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> Bf(cnt);
      HIPCHK(c, hipMemcpy(Bf.data(), c->Qw, cnt * 4, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < cnt; ++i) B[i] = Bf[i];
    }
    for (int l = 0; l < cfg.r; ++l)
      for (int64_t i = 0; i < cfg.n; ++i) V[(size_t)l * cfg.n + i] = B[(size_t)i * cfg.k + l];
  }
  if (d)
    for (int l = 0; l < cfg.r; ++l) d[l] = c->h_ctl->d[l];
  if (alpha) *alpha = c->h_ctl->alpha;
  if (t) *t = c->h_ctl->t;
  return MEG_OK;
}

meg_status meg_set_iterate(meg_ctx c, const double* V, int32_t q, const double* d, double alpha, int64_t t) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  const Cfg& cfg = c->cfg;
  if (!V || !d || q < 1 || q > cfg.r || !(alpha > 0.0) || t < 1) return MEG_ERR_INVALID_ARG;
  for (int l = 0; l < q; ++l)
    if (!(alpha + d[l] > 0.0)) return MEG_ERR_INVALID_ARG;
  for (int a = 0; a < q; ++a)
    for (int b = a; b < q; ++b) {
      double dot = 0.0;
      for (int64_t i = 0; i < cfg.n; ++i) dot += V[(size_t)a * cfg.n + i] * V[(size_t)b * cfg.n + i];
      if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-5) return MEG_ERR_INVALID_ARG;
    }
  return upload_iterate(c, V, q, d, alpha, t);
}

meg_status meg_get_state(meg_ctx c, void* buf, size_t* bytes) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!bytes) return MEG_ERR_INVALID_ARG;
  const size_t qbytes = (size_t)c->cfg.n * c->cfg.k * c->esize;
  const size_t need = 32 + sizeof(Ctl) + qbytes;
  if (!buf) {
    *bytes = need;
    return MEG_OK;
  }
  if (*bytes < need) return MEG_ERR_INVALID_ARG;
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  uint8_t* p = (uint8_t*)buf;
  uint32_t hdr[8] = {kStateMagic, 1u, (uint32_t)c->cfg.n, (uint32_t)(c->cfg.n >> 32), (uint32_t)c->cfg.k,
                     (uint32_t)c->cfg.r, (uint32_t)c->esize, (uint32_t)sizeof(Ctl)};
  std::memcpy(p, hdr, 32);
  std::memcpy(p + 32, c->h_ctl, sizeof(Ctl));
  HIPCHK(c, hipMemcpy(p + 32 + sizeof(Ctl), c->Qw, qbytes, hipMemcpyDeviceToHost));
  *bytes = need;
  return MEG_OK;
}

meg_status meg_set_state(meg_ctx c, const void* buf, size_t bytes) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  const size_t qbytes = (size_t)c->cfg.n * c->cfg.k * c->esize;
  const size_t need = 32 + sizeof(Ctl) + qbytes;
  if (!buf || bytes != need) return MEG_ERR_STATE;
  const uint8_t* p = (const uint8_t*)buf;
  uint32_t hdr[8];
  std::memcpy(hdr, p, 32);
  if (hdr[0] != kStateMagic || hdr[1] != 1u || hdr[2] != (uint32_t)c->cfg.n ||
      hdr[3] != (uint32_t)(c->cfg.n >> 32) || hdr[4] != (uint32_t)c->cfg.k || hdr[5] != (uint32_t)c->cfg.r ||
      hdr[6] != (uint32_t)c->esize || hdr[7] != (uint32_t)sizeof(Ctl))
    return MEG_ERR_STATE;
  std::memcpy(c->h_ctl, p + 32, sizeof(Ctl));
  HIPCHK(c, hipMemcpyAsync(c->ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->Qw, p + 32 + sizeof(Ctl), qbytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MEG_OK;
}

meg_status meg_profile_step(meg_ctx c, meg_kernel_times* out) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!out) return MEG_ERR_INVALID_ARG;
  const int ne = c->cfg.max_inner + 3;
  std::vector<hipEvent_t> ev(ne, nullptr);
  for (int i = 0; i < ne; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      return hip_fail(c);
    }
  dispatch<DoProfile>(c, ev.data());
  const bool ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(c->stream) == hipSuccess;
  std::memset(out, 0, sizeof(*out));
  float ms = 0.f;
  if (ok) {
    hipEventElapsedTime(&ms, ev[0], ev[1]);
    out->prep_ms = ms;
    for (int s = 1; s <= c->cfg.max_inner; ++s) {
      hipEventElapsedTime(&ms, ev[s], ev[s + 1]);
      out->sweep_ms[s - 1] = ms;
    }
    hipEventElapsedTime(&ms, ev[1 + c->cfg.max_inner], ev[2 + c->cfg.max_inner]);
    out->finalize_ms = ms;
    hipEventElapsedTime(&ms, ev[0], ev[2 + c->cfg.max_inner]);
    out->total_ms = ms;
    out->max_inner = c->cfg.max_inner;
  }
  for (auto e : ev) (void)hipEventDestroy(e);
  if (!ok) return hip_fail(c);
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  out->sweeps_active = c->h_ctl->info.inner_iters;
  return c->h_ctl->status ? (meg_status)c->h_ctl->status : MEG_OK;
}

void meg_destroy(meg_ctx c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_ctx(c);
}

}  // extern "C"
