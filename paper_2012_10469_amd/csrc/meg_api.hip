// Host runtime of the low-rank MEG library: the C ABI declared in include/meg.h.
//
// One context = one problem instance on one device stream.  The runtime
// validates arguments, allocates the device state, estimates the spectral
// bounds the solver's shift needs, builds the first iterate of Algorithm 2,
// and launches the persistent step kernel (meg_kernels.hpp) cooperatively:
// one launch runs one or many iterations with no host round trip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/meg.h"
#include "meg_host.hpp"
#include "meg_kernels.hpp"

using namespace meg;

// Device scratch of meg_dual_gap_static, for callers that cannot allocate:
// one file-scope array per GPU, held until the process ends.  Host code uses
// its device address from hipGetSymbolAddress (looked up per device at
// meg_init), never the array's name.
constexpr size_t kStaticScratchDoubles = (size_t)4 << 20;  // 32 MiB
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The current device's address of `scratch`, looked up once per device.
meg_status scratch_lookup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return MEG_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return MEG_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return MEG_ERR_DEVICE;
  }
  g_scratch[dev] = (double*)p;
  return MEG_OK;
}

constexpr uint32_t kStateMagic = 0x4d454731u;  // "MEG1"

constexpr int kStepNT = 512;                   // threads per persistent workgroup
constexpr int kMaxWgPerCu = 2;
constexpr int kMaxGrid = kBarGroupSize * kBarMaxGroups;  // barrier capacity
constexpr int kChunkSteps = 64;                // iterations per launch in meg_solve
constexpr int kTsSlots = kTsTotal;

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

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
  void* quad = nullptr;  // factored gradient scratch: y (L x k), K (L x L), w (L), ||a||^2 (L)
  Ctl* ctl = nullptr;
  double* part = nullptr;
  double* lz_prev = nullptr;  // the dual gap's last lambda_min Ritz vector (n doubles), its next start
  double* lz_ws = nullptr;    // Lanczos workspace of the gradient's lambda_min runs (kept, grown on demand)
  size_t lz_ws_doubles = 0;
  char* tr_ws = nullptr;      // the trace estimate's device buffers (kept, grown on demand)
  size_t tr_ws_bytes = 0;
  double* gpart = nullptr;
  double* sums = nullptr;
  unsigned* bar = nullptr;
  long long* ts = nullptr;
  size_t part_elems = 0;
  size_t cache_bytes = 0;  // dynamic LDS of the step kernel (CSR cache)
  // step-launch timing: a ring of HIP event pairs around each launch of the
  // step kernel, harvested (elapsed time summed) when the ring is full or the
  // counters are read
  static constexpr int kEvRing = 32;
  hipEvent_t ev_a[kEvRing] = {};
  hipEvent_t ev_b[kEvRing] = {};
  int ev_head = 0, ev_count = 0;
  double kernel_ms = 0.0;
  int64_t launches = 0;
  int64_t base_iters = 0, base_applies = 0, base_jacobi = 0, base_extrap = 0, base_unconv = 0;  // at the last reset
  int P = 1;               // persistent grid size
  int aux_nwg = 1;         // row-parallel auxiliary kernels
  Ctl* h_ctl = nullptr;    // pinned host mirror
  // pinned host words: the barrier error flag's copy, the stopping rule's
  // (tol, stop) and zeros for the asynchronous arm / disarm of meg_solve
  struct HostWords {
    unsigned bar_err;
    int32_t zero_i;
    double tol;
    double zero_d;
    int32_t stop;
  };
  HostWords* h_w = nullptr;
  bool external = false;   // the caller supplies G_t every step (meg_step_external)
  bool bilinear = false;   // bilinear measurements: the context forms G_t itself (external step path)
  void* bil_G = nullptr;   // bilinear: dense symmetric gradient n x n (state type, ld n)
  double* bil_res = nullptr;  // bilinear: residuals r_i (m)
  double* bil_P = nullptr;    // bilinear: per-slice partial gradients (bil_S x tile pairs x 64 x 64)
  int bil_S = 1;
  bool failed = false;
  int device = 0;  // the device current at meg_init
  bool da = false;         // dual-averaging reading (MEG_FLAG_DUAL_AVERAGE)
  void* da_Y = nullptr;    // its accumulated log-domain matrix Y (n x n, state type, ld n)
};

namespace {

meg_status hip_fail(meg_ctx c) {
  if (c) c->failed = true;
  return MEG_ERR_DEVICE;
}

#define HIPCHK(ctx, x)                           \
  do {                                           \
    if ((x) != hipSuccess) return hip_fail(ctx); \
  } while (0)

// ---------------------------------------------------------------------------
// launch helpers, dispatched on T (element type), KB (block size) and the
// operator family
// ---------------------------------------------------------------------------
// byte offsets of the factored-gradient scratch (one allocation)
struct QuadLayout {
  size_t y, k, w, na, bytes;
};
QuadLayout quad_layout(int64_t L, int k, size_t esize) {
  QuadLayout q;
  q.y = 0;
  q.k = (size_t)align16((int64_t)(L * k * esize));
  q.w = (size_t)align16((int64_t)(q.k + L * L * esize));
  q.na = q.w + (size_t)L * 8;
  q.bytes = q.na + (size_t)L * 8;
  return q;
}

template <typename T, int KB>
struct Launch {
  static bool x3(meg_ctx c) { return c->cfg.prec == MEG_PREC_F32_BF16X3; }
  static bool quad(meg_ctx c) { return c->cfg.kind == QUADMEAS; }
  static Data<T> data(meg_ctx c) {
    Data<T> d{};
    d.rp = c->obj.row_ptr;
    d.col = c->obj.col;
    d.val = (const T*)c->obj.val;
    if (x3(c)) {
      d.Dhi = (const uint16_t*)c->obj.dense;
      d.Dlo = (const uint16_t*)c->obj.dense_lo;
    } else {
      d.D = (const T*)c->obj.dense;
    }
    if (quad(c)) {
      const QuadLayout q = quad_layout(c->cfg.batch, c->cfg.k, sizeof(T));
      char* base = (char*)c->quad;
      d.A = (const T*)c->obj.A;
      d.bq = (const T*)c->obj.b;
      d.bidx = c->obj.batch_idx;
      d.qy = (T*)(base + q.y);
      d.qk = (T*)(base + q.k);
      d.qw = (double*)(base + q.w);
      d.qn = (double*)(base + q.na);
    }
    return d;
  }
  static DenseSrc<T> dense_src(meg_ctx c) {
    if (x3(c)) return DenseSrc<T>{nullptr, (const uint16_t*)c->obj.dense, (const uint16_t*)c->obj.dense_lo};
    return DenseSrc<T>{(const T*)c->obj.dense, nullptr, nullptr};
  }
  static bool csr(meg_ctx c) { return c->cfg.kind == LINEAR_CSR || c->cfg.kind == MASKED_CSR; }

  // step kernel of the context's operator family (the matrix-core form
  // exists for float state only, which validation guarantees)
  static const void* step_kernel(meg_ctx c) {
    if (csr(c)) return c->cfg.cache_blocks > 0 ? kernel<OP_CSR, true>() : kernel<OP_CSR>();
    if (quad(c)) return kernel<OP_FACTOR>();
    if constexpr (sizeof(T) == 4)
      if (x3(c)) return kernel<OP_DENSE_X3>();
    return kernel<OP_DENSE>();
  }
  static int rows_per_block(meg_ctx c) {
    if (csr(c)) return StepShape<T, KB, OP_CSR, kStepNT>::ROWS;
    if (quad(c)) return StepShape<T, KB, OP_FACTOR, kStepNT>::ROWS;
    if (x3(c)) return StepShape<T, KB, OP_DENSE_X3, kStepNT>::ROWS;
    return StepShape<T, KB, OP_DENSE, kStepNT>::ROWS;
  }

  template <int OPK, bool CACHE = false>
  static const void* kernel() {
    return reinterpret_cast<const void*>(&k_step<T, KB, OPK, kStepNT, CACHE>);
  }

  // Per-workgroup CSR cache in LDS: size it from the row pointers and enable
  // it when it fits beside the kernel's static LDS and keeps the grid
  // co-resident.  Sets cfg.cache_blocks / cache_nnz and c->cache_bytes.
  static void setup_cache(meg_ctx c) {
    Cfg& cfg = c->cfg;
    cfg.cache_blocks = 0;
    cfg.cache_nnz = 0;
    c->cache_bytes = 0;
    if (!csr(c) || (c->params.flags & MEG_FLAG_NO_LDS_CACHE)) return;
    constexpr int ROWS = StepShape<T, KB, OP_CSR, kStepNT>::ROWS;
    const int64_t n = cfg.n;
    std::vector<int32_t> rp((size_t)n + 1);
    if (hipMemcpy(rp.data(), c->obj.row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    const int64_t nblk = (n + ROWS - 1) / ROWS;
    int64_t max_nnz = 0;
    for (int w = 0; w < c->P; ++w) {
      int64_t cnt = 0;
      for (int64_t blk = w; blk < nblk; blk += c->P)
        cnt += rp[std::min<int64_t>(n, (blk + 1) * ROWS)] - rp[blk * ROWS];
      max_nnz = std::max(max_nnz, cnt);
    }
    const int blocks = (int)((nblk + c->P - 1) / c->P);
    const CacheLayout L = cache_layout(blocks, ROWS, (int)std::min<int64_t>(max_nnz, INT32_MAX), (int)sizeof(T),
                                       cfg.kind == MASKED_CSR);
    int dev = 0, lds_max = 0, ncu = 1, occ = 0;
    hipFuncAttributes fa{};
    const void* k = kernel<OP_CSR, true>();
    if (max_nnz > INT32_MAX / 4 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipFuncGetAttributes(&fa, k) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    if ((int64_t)fa.sharedSizeBytes + L.bytes > (int64_t)lds_max) return;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.bytes) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, kStepNT, (size_t)L.bytes) != hipSuccess ||
        (int64_t)ncu * occ < c->P) {
      (void)hipGetLastError();
      return;
    }
    cfg.cache_blocks = blocks;
    cfg.cache_nnz = (int)max_nnz;
    c->cache_bytes = (size_t)L.bytes;
  }

  // persistent grid: co-resident workgroups, no more than there are row blocks
  static int grid(meg_ctx c) {
    int dev = 0, ncu = 1, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void* k = step_kernel(c);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, kStepNT, 0) != hipSuccess || occ < 1) return 0;
    const int nblk = ceil_div(c->cfg.n, rows_per_block(c));
    return std::max(1, std::min(std::min(ncu * std::min(occ, kMaxWgPerCu), nblk), kMaxGrid));
  }

  static size_t part_need(int P) {
    // Gram partials, the objective's two partials and (FP64) the explicit
    // residuals' column sums
    return (size_t)P * ApplySmem<T, KB, 1, 0>::PSTRIDE;
  }

  static hipError_t step(meg_ctx c, int nsteps, bool stamps) {
    Cfg cfg = c->cfg;
    Ctl* ctl = c->ctl;
    Data<T> dat = data(c);
    T* Qw = (T*)c->Qw;
    T* Za = (T*)c->Za;
    T* Zb = (T*)c->Zb;
    T* g = (T*)c->g;
    Bufs b{c->part, c->gpart, c->sums, c->bar, stamps ? c->ts : nullptr};
    void* args[] = {&cfg, &ctl, &dat, &Qw, &Za, &Zb, &g, &b, &nsteps};
    return hipLaunchCooperativeKernel(step_kernel(c), dim3(c->P), dim3(kStepNT), args,
                                      cfg.cache_blocks > 0 ? c->cache_bytes : 0, c->stream);
  }

  // same grid as the step kernel (the barrier and partial buffers are sized for it)
  static hipError_t basis(meg_ctx c) {
    Cfg cfg = c->cfg;
    Ctl* ctl = c->ctl;
    T* Z0 = (T*)c->Qw;
    T* Z1 = (T*)c->Za;
    T* Z2 = (T*)c->Zb;
    Bufs b{c->part, c->gpart, c->sums, c->bar, nullptr};
    void* args[] = {&cfg, &ctl, &Z0, &Z1, &Z2, &b};
    const void* k = csr(c) ? reinterpret_cast<const void*>(&k_basis<T, KB, OP_CSR, kStepNT>)
                           : reinterpret_cast<const void*>(&k_basis<T, KB, OP_DENSE, kStepNT>);
    return hipLaunchCooperativeKernel(k, dim3(c->P), dim3(kStepNT), args, 0, c->stream);
  }

  // f(X_t): the basis is first written out explicitly (V = (B Wb)[:, :r])
  static hipError_t objective(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    const int nwg = ceil_div(cfg.n, 4);
    const int mwg = (int)std::min<int64_t>(4096, ceil_div(cfg.n * KB, 256));
    hipLaunchKernelGGL((k_materialize<T, KB>), dim3(mwg), dim3(256), 0, c->stream, cfg, c->ctl, (T*)c->Qw, (T*)c->Za,
                       (T*)c->Zb);
    if (quad(c)) {
      const int mb = sizeof(T) == 4 ? 4 : 2;  // measurements per wave (k_objective_quad)
      const int qwg = (int)std::min<int64_t>(c->aux_nwg, std::max<int64_t>(1, (cfg.m + 4 * mb - 1) / (4 * mb)));
      hipLaunchKernelGGL((k_objective_quad<T, KB>), dim3(qwg), dim3(256), 0, c->stream, cfg, c->ctl,
                         (const T*)c->obj.A, (const T*)c->obj.b, (const T*)c->Qw, (const T*)c->Za, (const T*)c->Zb,
                         c->part);
      hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c->stream, c->ctl, c->part, qwg, 0);
      return hipGetLastError();
    }
    if (csr(c))
      hipLaunchKernelGGL((k_objective_csr<T, KB>), dim3(nwg), dim3(256), 0, c->stream, cfg, c->ctl, c->obj.row_ptr,
                         c->obj.col, (const T*)c->obj.val, (const T*)c->Qw, (const T*)c->Za, (const T*)c->Zb,
                         c->part);
    else
      hipLaunchKernelGGL((k_objective_dense<T, KB>), dim3(nwg), dim3(256), 0, c->stream, cfg, c->ctl, dense_src(c),
                         (const T*)c->Qw, (const T*)c->Za, (const T*)c->Zb, c->part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c->stream, c->ctl, c->part, nwg, 0);
    return hipGetLastError();
  }

  // <X_t, grad f(X_t)> partials (one per group of 4 rows) into c->part, after
  // writing V out explicitly; masked: the gradient values into c->g
  static hipError_t xdotg(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    const int nwg = ceil_div(cfg.n, 4);
    const int mwg = (int)std::min<int64_t>(4096, ceil_div(cfg.n * KB, 256));
    hipLaunchKernelGGL((k_materialize<T, KB>), dim3(mwg), dim3(256), 0, c->stream, cfg, c->ctl, (T*)c->Qw, (T*)c->Za,
                       (T*)c->Zb);
    if (csr(c))
      hipLaunchKernelGGL((k_xdotg_csr<T, KB>), dim3(nwg), dim3(256), 0, c->stream, cfg, c->ctl, c->obj.row_ptr,
                         c->obj.col, (const T*)c->obj.val, (T*)c->g, (const T*)c->Qw, (const T*)c->Za,
                         (const T*)c->Zb, c->part);
    else
      hipLaunchKernelGGL((k_xdotg_dense<T, KB>), dim3(nwg), dim3(256), 0, c->stream, cfg, c->ctl, dense_src(c),
                         (const T*)c->Qw, (const T*)c->Za, (const T*)c->Zb, c->part);
    return hipGetLastError();
  }

  // bilinear measurements at the current iterate: residuals and f(X_t)
  // (ctl->f), then, when `grad`, the dense symmetric gradient into c->bil_G
  static hipError_t bilinear(meg_ctx c, bool grad) {
    const Cfg& cfg = c->cfg;
    const int64_t n = cfg.n, m = c->obj.m;
    const int p = std::max(1, (int)c->obj.batch);  // columns per measurement matrix
    const int mwg = (int)std::min<int64_t>(4096, ceil_div(n * KB, 256));
    hipLaunchKernelGGL((k_materialize<T, KB>), dim3(mwg), dim3(256), 0, c->stream, cfg, c->ctl, (T*)c->Qw, (T*)c->Za,
                       (T*)c->Zb);
    const int rg = (int)std::min<int64_t>(1024, ceil_div(m, 4));
    // V staged in LDS when it fits in 48 KB (read from the basis otherwise)
    const size_t vbytes = (size_t)cfg.r * (size_t)n * sizeof(T);
    const int qlds = vbytes <= 48 * 1024 ? 1 : 0;
    hipLaunchKernelGGL((k_bil_resid<T, KB>), dim3(rg), dim3(256), qlds ? vbytes : 0, c->stream, cfg,
                       (const Ctl*)c->ctl, (const T*)c->Qw, (const T*)c->Za, (const T*)c->Zb, (const T*)c->obj.A,
                       c->obj.lda, (const T*)c->obj.b, m, p, c->bil_res, c->part, qlds);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c->stream, c->ctl, c->part, rg, 0);
    if (grad) {
      const int tiles = (int)ceil_div(n, kBilTile), pairs = tiles * (tiles + 1) / 2;
      const int64_t rows = m * p;
      const int64_t per = ceil_div(ceil_div(rows, c->bil_S), 16) * 16;
      hipLaunchKernelGGL((k_bil_grad_part<T>), dim3(pairs, 1, c->bil_S), dim3(256), 0, c->stream, n,
                         (const T*)c->obj.A, c->obj.lda, rows, p, (const double*)c->bil_res, per, tiles, c->bil_P);
      const int64_t cells = (int64_t)pairs * kBilTile * kBilTile;
      const int sg = (int)std::max<int64_t>(1, std::min<int64_t>(8192, ceil_div(cells, 256)));
      hipLaunchKernelGGL((k_bil_grad_sum<T>), dim3(sg), dim3(256), 0, c->stream, n, c->bil_S, pairs, tiles,
                         (const double*)c->bil_P, (T*)c->bil_G);
    }
    return hipGetLastError();
  }

  // dual-averaging reading: Y = log X_t of the current iterate
  static hipError_t da_init(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    const int mwg = (int)std::min<int64_t>(4096, ceil_div(cfg.n * KB, 256));
    hipLaunchKernelGGL((k_materialize<T, KB>), dim3(mwg), dim3(256), 0, c->stream, cfg, c->ctl, (T*)c->Qw, (T*)c->Za,
                       (T*)c->Zb);
    hipLaunchKernelGGL((k_da_init<T, KB>), dim3(cfg.n), dim3(256), 0, c->stream, cfg, (const Ctl*)c->ctl,
                       (const T*)c->Qw, (const T*)c->Za, (const T*)c->Zb, (T*)c->da_Y);
    return hipGetLastError();
  }
  // Y <- Y - eta grad f(X_t), its Gershgorin bounds, then the step's shift
  // and coefficients for Y + sigma' I
  static hipError_t da_update(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    const int mwg = (int)std::min<int64_t>(4096, ceil_div(cfg.n * KB, 256));
    hipLaunchKernelGGL((k_materialize<T, KB>), dim3(mwg), dim3(256), 0, c->stream, cfg, c->ctl, (T*)c->Qw, (T*)c->Za,
                       (T*)c->Zb);
    hipLaunchKernelGGL((k_da_update<T, KB>), dim3(cfg.n), dim3(256), 0, c->stream, cfg, (const Ctl*)c->ctl,
                       (const T*)c->obj.dense, (const T*)c->Qw, (const T*)c->Za, (const T*)c->Zb, (T*)c->da_Y,
                       c->part);
    hipLaunchKernelGGL(k_da_setup, dim3(1), dim3(64), 0, c->stream, cfg, c->ctl, (const double*)c->part,
                       (int)cfg.n);
    return hipGetLastError();
  }

  static hipError_t data_norm(meg_ctx c) {
    const Cfg& cfg = c->cfg;
    int64_t rows, cols, ld;
    DenseSrc<T> x;
    if (!csr(c)) {
      rows = cfg.n; cols = cfg.n; ld = cfg.ld; x = dense_src(c);
    } else {
      rows = cfg.nnz > 0 ? 1 : 0; cols = std::max<int64_t>(cfg.nnz, 1); ld = 0;
      x = DenseSrc<T>{(const T*)c->obj.val, nullptr, nullptr};
    }
    const int64_t total = rows * cols;
    const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (total + 255) / 256));
    hipLaunchKernelGGL((k_sumsq<T>), dim3(nwg), dim3(256), 0, c->stream, x, rows, cols, ld, c->part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c->stream, c->ctl, c->part, nwg, 1);
    return hipGetLastError();
  }
};

template <template <typename, int> class F, typename... Args>
auto dispatch(meg_ctx c, Args&&... args) {
  const bool dbl = c->esize == 8;
  if (c->cfg.k == 16) return dbl ? F<double, 16>::run(c, args...) : F<float, 16>::run(c, args...);
  return dbl ? F<double, 32>::run(c, args...) : F<float, 32>::run(c, args...);
}

template <typename T, int KB> struct DoStep {
  static hipError_t run(meg_ctx c, int nsteps, bool st) { return Launch<T, KB>::step(c, nsteps, st); }
};
template <typename T, int KB> struct DoBasis {
  static hipError_t run(meg_ctx c) { return Launch<T, KB>::basis(c); }
};
template <typename T, int KB> struct DoObjective {
  static hipError_t run(meg_ctx c) { return Launch<T, KB>::objective(c); }
};
template <typename T, int KB> struct DoNorm {
  static hipError_t run(meg_ctx c) { return Launch<T, KB>::data_norm(c); }
};
template <typename T, int KB> struct DoGrid {
  static int run(meg_ctx c) { return Launch<T, KB>::grid(c); }
};
template <typename T, int KB> struct DoCache {
  static int run(meg_ctx c) {
    Launch<T, KB>::setup_cache(c);
    return 0;
  }
};
template <typename T, int KB> struct DoXdotG {
  static hipError_t run(meg_ctx c) { return Launch<T, KB>::xdotg(c); }
};
template <typename T, int KB> struct DoBilinear {
  static hipError_t run(meg_ctx c, bool grad) { return Launch<T, KB>::bilinear(c, grad); }
};
template <typename T, int KB> struct DoDaInit {
  static hipError_t run(meg_ctx c) { return Launch<T, KB>::da_init(c); }
};
template <typename T, int KB> struct DoDaUpdate {
  static hipError_t run(meg_ctx c) { return Launch<T, KB>::da_update(c); }
};
template <typename T, int KB> struct DoPartNeed {
  static size_t run(meg_ctx c, int P) { return Launch<T, KB>::part_need(P); }
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
    if (hipMemcpy(dx, xt.data(), n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
      st = hip_fail(c);
      break;
    }
    hipLaunchKernelGGL((k_matvec<T>), dim3(ceil_div(n, 4)), dim3(256), 0, c->stream, cfg, Launch<T, 16>::dense_src(c),
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

// n x k block i (0, 1, 2) of the context
void* block(meg_ctx c, int i) { return i == 0 ? c->Qw : (i == 1 ? c->Za : c->Zb); }

meg_status copy_ctl_to_host(meg_ctx c) {
  HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MEG_OK;
}

// The control block and the barrier's error flag copied to the host with
// one synchronisation; MEG_ERR_DEVICE when a grid barrier did not complete.
meg_status sync_ctl(meg_ctx c) {
  HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&c->h_w->bar_err, c->bar + kBarErr, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->h_w->bar_err) return hip_fail(c);
  return MEG_OK;
}

// Workspace of a Lanczos run for the smallest eigenvalue of the gradient,
// in doubles: the basis V ((m + 1) x n), y, w and the product input x (n
// each; x holds n elements of the state's type), reorthogonalisation
// coefficients h (m + 1), alpha/beta ab (2m), deflation coefficients lp (KMAX).
struct LzWs {
  double *V, *y, *w, *x, *h, *ab, *lp;
};
int lz_steps(int64_t n, int defl, int max_steps) { return (int)std::min<int64_t>(n - defl, max_steps); }
size_t lz_ws_need(int64_t n, int m) {
  return (size_t)(m + 1) * n + 3 * (size_t)n + (size_t)(m + 1) + 2 * (size_t)m + KMAX;
}
LzWs lz_ws_carve(double* base, int64_t n, int m) {
  LzWs ws;
  ws.V = base;
  ws.y = ws.V + (size_t)(m + 1) * n;
  ws.w = ws.y + n;
  ws.x = ws.w + n;
  ws.h = ws.x + n;
  ws.ab = ws.h + (m + 1);
  ws.lp = ws.ab + 2 * (size_t)m;
  return ws;
}

// Smallest eigenvalue of the gradient G = grad f(X_t) by Lanczos with full
// reorthogonalisation (two classical Gram-Schmidt passes).  The basis, the
// recurrence and the products with G run on the device (products: k_matvec
// with C, M, or the pattern holding the gradient values xdotg wrote into
// c->g; denoising adds alpha x + V diag(d) V^T x from the materialised
// basis); the host only draws the start vector and, every 8 steps, solves
// the small tridiagonal eigenproblem for the convergence test.
// defl > 0: the run is restricted to the orthogonal complement of the first
// defl columns of the materialised basis (the iterate's V): the start vector
// and every new vector are orthogonalised against them too, so the result is
// lambda_min of G on that complement.  warm: start from (and keep) the
// context's previous lambda_min Ritz vector (plain runs only).
template <typename T>
meg_status lanczos_grad_min(meg_ctx c, int max_steps, double tol, const LzWs& ws, int defl, bool warm,
                            meg_dual_gap_info* out) {
  const Cfg& cfg = c->cfg;
  const int64_t n = cfg.n;
  const int r = cfg.r, KB = cfg.k;
  const int m = lz_steps(n, defl, max_steps);
  const bool den = cfg.kind == DENOISE_DENSE;
  const bool masked = cfg.kind == MASKED_CSR;
  const T* Qm = (const T*)block(c, (c->h_ctl->src + 1) % 3);  // materialised basis (xdotg)
  double *V = ws.V, *y = ws.y, *w = ws.w, *h = ws.h, *ab = ws.ab, *lp = ws.lp;
  T* xt = (T*)ws.x;
  if (m < 1) return MEG_ERR_INVALID_ARG;
  // start vector: the previous call's lambda_min Ritz vector (the gradient
  // changes little between nearby iterates) plus 1e-3 of a seeded Gaussian
  // vector, or the Gaussian vector alone; normalised on the host
  std::vector<double> v0(n);
  SplitMix rng{c->params.seed ^ 0x6475616c67617021ull ^ (uint64_t)c->h_ctl->t ^ ((uint64_t)defl << 40)};
  for (int64_t i = 0; i < n; ++i) v0[i] = rng.normal();
  if (warm && c->lz_prev) {
    std::vector<double> u(n);
    if (hipMemcpy(u.data(), c->lz_prev, n * 8, hipMemcpyDeviceToHost) != hipSuccess) return hip_fail(c);
    double gn = 0.0;
    for (int64_t i = 0; i < n; ++i) gn += v0[i] * v0[i];
    gn = std::sqrt(gn);
    for (int64_t i = 0; i < n; ++i) v0[i] = u[i] + 1e-3 * v0[i] / gn;
  }
  double nrm = 0.0;
  for (int64_t i = 0; i < n; ++i) nrm += v0[i] * v0[i];
  nrm = std::sqrt(nrm);
  for (int64_t i = 0; i < n; ++i) v0[i] /= nrm;
  meg_status st = MEG_OK;
  std::vector<double> abh(2 * (size_t)m), smin;
  double theta = 0.0, res = 0.0;
  int done = 0;
  bool conv = false;
  const int gv = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256));
  const hipStream_t sm = c->stream;
  // w <- w - Q[:, :defl] (Q[:, :defl]^T w), twice
  auto deflate = [&](double* vec) {
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL((k_lz_defl_dots<T>), dim3(defl), dim3(256), 0, sm, Qm, KB, (const double*)vec, n, lp);
      hipLaunchKernelGGL((k_lz_defl_sub<T>), dim3(gv), dim3(256), 0, sm, Qm, KB, defl, (const double*)lp, n, vec);
    }
  };
  if (defl > 0) {
    if (hipMemcpyAsync(w, v0.data(), n * 8, hipMemcpyHostToDevice, sm) != hipSuccess) st = hip_fail(c);
    deflate(w);
    hipLaunchKernelGGL(k_lz_unit, dim3(1), dim3(256), 0, sm, (const double*)w, n, V);
  } else if (hipMemcpyAsync(V, v0.data(), n * 8, hipMemcpyHostToDevice, sm) != hipSuccess) {
    st = hip_fail(c);
  }
  for (int j = 0; st == MEG_OK && j < m; ++j) {
    const double* vj = V + (int64_t)j * n;
    // y = G v_j
    hipLaunchKernelGGL((k_lz_cast<T>), dim3(gv), dim3(256), 0, sm, vj, n, xt);
    hipLaunchKernelGGL((k_matvec<T>), dim3(ceil_div(n, 4)), dim3(256), 0, sm, cfg, Launch<T, 16>::dense_src(c),
                       c->obj.row_ptr, c->obj.col, masked ? (const T*)c->g : (const T*)c->obj.val, (const T*)xt, y);
    if (den) {
      hipLaunchKernelGGL((k_lz_lr_dots<T>), dim3(r), dim3(256), 0, sm, Qm, KB, (const T*)xt, n, lp);
      hipLaunchKernelGGL((k_lz_lr_update<T>), dim3(gv), dim3(256), 0, sm, (const Ctl*)c->ctl, Qm, KB, r,
                         (const T*)xt, (const double*)lp, n, y);
    }
    // alpha_j, the three-term recurrence, two reorthogonalisation passes
    // (and the deflation), beta_j and v_{j+1}
    hipLaunchKernelGGL(k_lz_dots, dim3(1), dim3(256), 0, sm, vj, (const double*)y, n, ab + j);
    hipLaunchKernelGGL(k_lz_three_term, dim3(gv), dim3(256), 0, sm, (const double*)V, (const double*)y,
                       (const double*)ab, j, m, n, w);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_lz_dots, dim3(j + 1), dim3(256), 0, sm, (const double*)V, (const double*)w, n, h);
      hipLaunchKernelGGL(k_lz_sub, dim3(gv), dim3(256), 0, sm, (const double*)V, (const double*)h, j + 1, n, w);
    }
    if (defl > 0) deflate(w);
    hipLaunchKernelGGL(k_lz_next, dim3(1), dim3(256), 0, sm, (const double*)w, j, m, n, ab, V);
    if (hipGetLastError() != hipSuccess) {
      st = hip_fail(c);
      break;
    }
    done = j + 1;
    if (done % 8 != 0 && done != m) continue;
    if (hipMemcpyAsync(abh.data(), ab, abh.size() * 8, hipMemcpyDeviceToHost, sm) != hipSuccess ||
        hipStreamSynchronize(sm) != hipSuccess) {
      st = hip_fail(c);
      break;
    }
    // the Krylov space is invariant at the first vanishing beta
    int j1 = done;
    bool invariant = false;
    for (int q = 0; q < done; ++q)
      if (abh[m + q] == 0.0) {
        j1 = q + 1;
        invariant = true;
        break;
      }
    std::vector<double> Tm((size_t)j1 * j1, 0.0), ev, S;
    for (int q = 0; q < j1; ++q) {
      Tm[(size_t)q * j1 + q] = abh[q];
      if (q + 1 < j1) Tm[(size_t)q * j1 + q + 1] = Tm[(size_t)(q + 1) * j1 + q] = abh[m + q];
    }
    host_sym_eig(Tm, j1, ev, S);
    int imin = 0;
    double scale = 0.0;
    for (int q = 0; q < j1; ++q) {
      if (ev[q] < ev[imin]) imin = q;
      scale = std::max(scale, std::fabs(ev[q]));
    }
    theta = ev[imin];
    res = std::fabs(abh[m + j1 - 1] * S[(size_t)(j1 - 1) * j1 + imin]);
    conv = res <= tol * scale;
    done = j1;
    smin.assign(j1, 0.0);
    for (int q = 0; q < j1; ++q) smin[q] = S[(size_t)q * j1 + imin];
    if (conv || invariant) break;
  }
  // keep the Ritz vector V s of lambda_min for the next call's start
  if (st == MEG_OK && warm && !smin.empty()) {
    if (!c->lz_prev && hipMalloc((void**)&c->lz_prev, std::max<size_t>(n * 8, 256)) != hipSuccess) {
      (void)hipGetLastError();
      c->lz_prev = nullptr;  // no warm start next time; not an error
    }
    if (c->lz_prev) {
      if (hipMemcpyAsync(h, smin.data(), smin.size() * 8, hipMemcpyHostToDevice, sm) != hipSuccess) {
        st = hip_fail(c);
      } else {
        hipLaunchKernelGGL(k_lz_combine, dim3(gv), dim3(256), 0, sm, (const double*)V, (const double*)h,
                           (int)smin.size(), n, c->lz_prev);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(sm) != hipSuccess) st = hip_fail(c);
      }
    }
  }
  if (st == MEG_OK && hipStreamSynchronize(sm) != hipSuccess) st = hip_fail(c);
  if (st != MEG_OK) return st;
  out->lambda_min = theta;
  out->resid = res;
  out->steps = done;
  out->converged = conv ? 1 : 0;
  return MEG_OK;
}

// meg_dual_gap_static's workspace: the context's device's copy of `scratch`.
meg_status static_scratch(meg_ctx c, double** base) {
  double* p = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch[c->device] : nullptr;
  if (!p) return MEG_ERR_DEVICE;
  *base = p;
  return MEG_OK;
}

// The context's Lanczos workspace for m steps: allocated on first use and
// kept (grown when a later call needs more), so repeated calls allocate
// nothing.
meg_status ctx_lz_ws(meg_ctx c, int m, LzWs* ws) {
  const size_t need = lz_ws_need(c->cfg.n, m);
  if (need > c->lz_ws_doubles) {
    if (c->lz_ws) (void)hipFree(c->lz_ws);
    c->lz_ws = nullptr;
    c->lz_ws_doubles = 0;
    if (hipMalloc((void**)&c->lz_ws, need * 8) != hipSuccess) {
      (void)hipGetLastError();
      c->lz_ws = nullptr;
      return MEG_ERR_OUT_OF_MEMORY;
    }
    c->lz_ws_doubles = need;
  }
  *ws = lz_ws_carve(c->lz_ws, c->cfg.n, m);
  return MEG_OK;
}

// Eigenvalues of the symmetric tridiagonal T (diagonal a[0..m), off-diagonal
// b[0..m-1)) and the first components z of its unit eigenvectors, by implicit
// QR steps with Wilkinson's shift on the trailing unreduced block (Golub and
// Van Loan, Matrix Computations, Section 8.3), accumulating only the first
// column of the rotation product.  These are the nodes and weights z_i^2 of
// the Gauss quadrature of the Lanczos run (Golub and Welsch).  a and b are
// destroyed; a returns the eigenvalues.
void tridiag_eig_first(std::vector<double>& a, std::vector<double>& b, std::vector<double>& z) {
  const int m = (int)a.size();
  z.assign(m, 0.0);
  if (m == 0) return;
  z[0] = 1.0;
  double tnorm = 0.0;
  for (int i = 0; i < m; ++i)
    tnorm = std::max(tnorm, std::fabs(a[i]) + (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0));
  auto negligible = [&](int i) {
    return std::fabs(b[i]) <= 2.3e-16 * (std::fabs(a[i]) + std::fabs(a[i + 1])) || std::fabs(b[i]) <= 1e-18 * tnorm;
  };
  int hi = m - 1, iters = 0;
  while (hi > 0 && iters < 60 * m) {
    if (negligible(hi - 1)) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !negligible(lo - 1)) --lo;
    if (lo > 0) b[lo - 1] = 0.0;
    ++iters;
    // shift: the eigenvalue of the trailing 2 x 2 block nearer to a[hi]
    const double d = 0.5 * (a[hi - 1] - a[hi]), e = b[hi - 1];
    const double mu = a[hi] - e * (e / (d + std::copysign(std::hypot(d, e), d)));
    // one QR step on rows lo..hi: rotation k acts on rows/columns k, k + 1,
    // zeroing the bulge (k + 1, k - 1) the previous rotation left
    double x = a[lo] - mu, y = b[lo];
    for (int k = lo; k < hi; ++k) {
      const double rr = std::hypot(x, y);
      const double c = rr > 0.0 ? x / rr : 1.0, s = rr > 0.0 ? y / rr : 0.0;
      if (k > lo) b[k - 1] = rr;
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      const double zk = z[k], zk1 = z[k + 1];
      z[k] = c * zk + s * zk1;
      z[k + 1] = c * zk1 - s * zk;
      if (k + 1 < hi) {
        x = b[k];
        y = s * b[k + 1];
        b[k + 1] *= c;
      }
    }
  }
}

// log(e_1^T exp(T) e_1) = log sum_i z_i^2 exp(theta_i) for the tridiagonal T
// with diagonal a and off-diagonal b (copies)
double log_quad_exp(std::vector<double> a, std::vector<double> b) {
  std::vector<double> z;
  tridiag_eig_first(a, b, z);
  double mx = -std::numeric_limits<double>::infinity();
  for (size_t i = 0; i < a.size(); ++i)
    if (z[i] != 0.0) mx = std::max(mx, a[i] + 2.0 * std::log(std::fabs(z[i])));
  if (!std::isfinite(mx)) return mx;
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i)
    if (z[i] != 0.0) s += std::exp(a[i] + 2.0 * std::log(std::fabs(z[i])) - mx);
  return mx + std::log(s);
}

double log_sum_exp(const std::vector<double>& v) {
  double mx = -std::numeric_limits<double>::infinity();
  for (double x : v) mx = std::max(mx, x);
  if (!std::isfinite(mx)) return mx;
  double s = 0.0;
  for (double x : v) s += std::exp(x - mx);
  return mx + std::log(s);
}

// Cholesky G = R^T R of the kq x kq Gram matrix G[l * 64 + b] with columns
// whose remaining pivot is <= 1e-12 of the largest diagonal dropped (their row
// and column of R^{-1} are zero); Rinv (64 x 64, row-major) = R^{-1}.
// Returns the number of columns kept.
int chol_inv_drop(const std::vector<double>& G, int kq, std::vector<double>& Rinv) {
  std::vector<double> R((size_t)kq * kq, 0.0);
  std::vector<char> keep(kq, 0);
  double dmax = 0.0;
  for (int j = 0; j < kq; ++j) dmax = std::max(dmax, G[(size_t)j * kTrW + j]);
  int kept = 0;
  for (int j = 0; j < kq; ++j) {
    double dj = G[(size_t)j * kTrW + j];
    for (int l = 0; l < j; ++l)
      if (keep[l]) dj -= R[(size_t)l * kq + j] * R[(size_t)l * kq + j];
    if (!(dj > 1e-12 * dmax)) continue;
    keep[j] = 1;
    ++kept;
    const double rjj = std::sqrt(dj);
    R[(size_t)j * kq + j] = rjj;
    for (int c = j + 1; c < kq; ++c) {
      double v = G[(size_t)j * kTrW + c];
      for (int l = 0; l < j; ++l)
        if (keep[l]) v -= R[(size_t)l * kq + j] * R[(size_t)l * kq + c];
      R[(size_t)j * kq + c] = v / rjj;
    }
  }
  // R X = I on the kept indices, by back substitution per column
  Rinv.assign((size_t)kTrW * kTrW, 0.0);
  for (int c = 0; c < kq; ++c) {
    if (!keep[c]) continue;
    for (int i = c; i >= 0; --i) {
      if (!keep[i]) continue;
      double s = (i == c) ? 1.0 : 0.0;
      for (int l = i + 1; l <= c; ++l)
        if (keep[l]) s -= R[(size_t)i * kq + l] * Rinv[(size_t)l * kTrW + c];
      Rinv[(size_t)i * kTrW + c] = s / R[(size_t)i * kq + i];
    }
  }
  return kept;
}

// out[l * 64 + b] = sum_i A[i * lda + l] X[i][b] (l < na) and out[b] =
// sum_i A[i][b] B[i][b]: partial sums over G workgroups, then their sum in order
template <typename TA>
void tr_gram(hipStream_t sm, const TA* A, int64_t lda, int na, const double* X, int64_t n, int G, double* part,
             double* out) {
  hipLaunchKernelGGL((k_tr_gram_part<TA>), dim3(G), dim3(256), 0, sm, A, lda, na, X, n, part);
  hipLaunchKernelGGL(k_tr_part_sum, dim3(ceil_div(na * kTrW, 4)), dim3(256), 0, sm, (const double*)part, G,
                     na * kTrW, out);
}
void tr_cdot(hipStream_t sm, const double* A, const double* B, int64_t n, int G, double* part, double* out) {
  hipLaunchKernelGGL(k_tr_cdot_part, dim3(G), dim3(256), 0, sm, A, B, n, part);
  hipLaunchKernelGGL(k_tr_part_sum, dim3(kTrW / 4), dim3(256), 0, sm, (const double*)part, G, kTrW, out);
}

// The deflated probe estimate of tr exp(M_t) (see meg_trace_exp).  Up to 64
// vectors per lockstep Lanczos batch: batch 0 holds the orthonormalised block
// columns and the first probes, later batches 64 probes each.
template <typename T>
meg_status trace_exp_run(meg_ctx c, const double* probes, int p, double weight, int max_steps, double tol,
                         meg_trace_info* out) {
  const Cfg& cfg = c->cfg;
  const int64_t n = cfg.n;
  const int r = cfg.r, KB = cfg.k;
  const int kq = (int)std::min<int64_t>(KB, n);
  const int m = (int)std::min<int64_t>(max_steps, n);
  const bool den = cfg.kind == DENOISE_DENSE, masked = cfg.kind == MASKED_CSR;
  const bool csr = masked || cfg.kind == LINEAR_CSR;
  const T* Qm = (const T*)block(c, (c->h_ctl->src + 1) % 3);  // materialised basis (xdotg)
  // M_t x = s Op x + c0 x + V diag(cv) V^T x: log X_t = log(alpha) I +
  // V diag(log(alpha + d) - log alpha) V^T, and -eta G with G = C (linear),
  // X_t - M (denoising) or the gradient values on the pattern (masked)
  const Ctl& h = *c->h_ctl;
  const double la = std::log(h.alpha);
  double c0 = la, sop = -cfg.eta;
  std::vector<double> cv(KMAX, 0.0);
  for (int l = 0; l < r; ++l) cv[l] = std::log(h.alpha + h.d[l]) - la;
  if (den) {
    c0 = la - cfg.eta * h.alpha;
    sop = cfg.eta;
    for (int l = 0; l < r; ++l) cv[l] -= cfg.eta * h.d[l];
  }
  const size_t vbytes = (size_t)n * kTrW * 8;
  double *Qd = nullptr, *B0 = nullptr, *B1 = nullptr, *B2 = nullptr, *Y = nullptr, *al = nullptr, *bb = nullptr;
  double *P = nullptr, *Mx = nullptr, *dcv = nullptr, *sm1 = nullptr, *sm2 = nullptr, *part = nullptr;
  const int GR = (int)std::min<int64_t>(kTrRedWG, ceil_div(n, 4));
  // the buffers are carved from one context workspace, allocated on first
  // use and kept (grown when a later call needs more): repeated calls
  // allocate nothing
  double** bufs[] = {&Qd, &B0, &B1, &B2, &Y, &al, &bb, &P, &Mx, &dcv, &sm1, &sm2, &part};
  const size_t sizes[] = {vbytes, vbytes, vbytes, vbytes, vbytes, (size_t)m * kTrW * 8, (size_t)m * kTrW * 8,
                          (size_t)kTrW * kTrW * 8, (size_t)kTrW * kTrW * 8, (size_t)KMAX * 8, (size_t)kTrW * 8,
                          (size_t)kTrW * 8, (size_t)GR * 32 * kTrW * 8};
  size_t need = 0;
  for (size_t b : sizes) need += (b + 255) / 256 * 256;
  if (need > c->tr_ws_bytes) {
    if (c->tr_ws) (void)hipFree(c->tr_ws);
    c->tr_ws = nullptr;
    c->tr_ws_bytes = 0;
    if (hipMalloc((void**)&c->tr_ws, need) != hipSuccess) {
      (void)hipGetLastError();
      c->tr_ws = nullptr;
      return MEG_ERR_OUT_OF_MEMORY;
    }
    c->tr_ws_bytes = need;
  }
  {
    size_t off = 0;
    for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); ++i) {
      *bufs[i] = reinterpret_cast<double*>(c->tr_ws + off);
      off += (sizes[i] + 255) / 256 * 256;
    }
  }
  const hipStream_t sm = c->stream;
  const int ge = (int)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(n * kTrW, 256)));
  const int gw = ceil_div(n, 4);
  meg_status st = MEG_OK;
  auto fail = [&]() {
    st = hip_fail(c);
    return st;
  };
  if (hipMemcpyAsync(dcv, cv.data(), KMAX * 8, hipMemcpyHostToDevice, sm) != hipSuccess) return fail();
  // orthonormal FP64 deflation basis: the block's kq columns, Cholesky QR twice
  hipLaunchKernelGGL((k_tr_load<T>), dim3(ge), dim3(256), 0, sm, Qm, KB, (const double*)nullptr, kq,
                     (const double*)nullptr, 0, n, Qd);
  int kd = kq;
  std::vector<double> Gh((size_t)kTrW * kTrW), Rinv;
  for (int pass = 0; pass < 2 && kq > 0; ++pass) {
    tr_gram<double>(sm, Qd, kTrW, kq, Qd, n, GR, part, P);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(Gh.data(), P, (size_t)kq * kTrW * 8, hipMemcpyDeviceToHost, sm) != hipSuccess ||
        hipStreamSynchronize(sm) != hipSuccess)
      return fail();
    kd = chol_inv_drop(Gh, kq, Rinv);
    if (hipMemcpyAsync(Mx, Rinv.data(), (size_t)kTrW * kTrW * 8, hipMemcpyHostToDevice, sm) != hipSuccess)
      return fail();
    hipLaunchKernelGGL(k_tr_rowmix, dim3(gw), dim3(256), 0, sm, (const double*)Qd, (const double*)Mx, kq, 0, kq, 0,
                       n, Qd);
  }
  std::vector<double> defl, tail(p, -std::numeric_limits<double>::infinity());
  std::vector<double> abh((size_t)m * kTrW), bbh((size_t)m * kTrW), nsq(kTrW), nsq0(kTrW), sc(kTrW);
  bool all_conv = true;
  int max_done = 0, batches = 0;
  int next_probe = 0;
  for (int batch = 0; batch == 0 || next_probe < p; ++batch) {
    const int nq = batch == 0 ? kq : 0;
    const int np_b = std::min(p - next_probe, kTrW - nq);
    ++batches;
    // start vectors: block columns, then the probes projected by I - Qd Qd^T
    // (two passes), then normalised
    hipLaunchKernelGGL((k_tr_load<T>), dim3(ge), dim3(256), 0, sm, (const T*)nullptr, KB, (const double*)Qd, nq,
                       np_b > 0 ? probes + (int64_t)next_probe * n : (const double*)nullptr, np_b, n, B0);
    tr_cdot(sm, B0, B0, n, GR, part, sm2);
    for (int pass = 0; pass < 2 && kq > 0 && np_b > 0; ++pass) {
      tr_gram<double>(sm, Qd, kTrW, kq, B0, n, GR, part, P);
      hipLaunchKernelGGL(k_tr_rowmix, dim3(gw), dim3(256), 0, sm, (const double*)Qd, (const double*)P, kq, nq,
                         nq + np_b, 1, n, B0);
    }
    tr_cdot(sm, B0, B0, n, GR, part, sm1);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(nsq0.data(), sm2, kTrW * 8, hipMemcpyDeviceToHost, sm) != hipSuccess ||
        hipMemcpyAsync(nsq.data(), sm1, kTrW * 8, hipMemcpyDeviceToHost, sm) != hipSuccess ||
        hipStreamSynchronize(sm) != hipSuccess)
      return fail();
    // a probe the projection reduced to rounding error lies in span(Q): zero
    for (int b = 0; b < kTrW; ++b) {
      if (!(nsq[b] > 1e-26 * nsq0[b]) || !(nsq[b] > 1e-300)) nsq[b] = 0.0;
      sc[b] = nsq[b] > 0.0 ? 1.0 / std::sqrt(nsq[b]) : 0.0;
    }
    if (hipMemcpyAsync(sm2, sc.data(), kTrW * 8, hipMemcpyHostToDevice, sm) != hipSuccess) return fail();
    hipLaunchKernelGGL(k_tr_scale, dim3(ge), dim3(256), 0, sm, (const double*)sm2, n, B0);
    // lockstep Lanczos: Xc the current vectors, Xp the previous ones
    double *Xp = B2, *Xc = B0, *Wn = B1;
    std::vector<double> lq(kTrW, -std::numeric_limits<double>::infinity()), lq_prev(kTrW);
    std::vector<char> conv(kTrW, 0);
    bool batch_conv = false;
    int done = 0;
    for (int j = 0; j < m; ++j) {
      if (csr)
        hipLaunchKernelGGL((k_tr_matvec_csr<T>), dim3(gw), dim3(256), 0, sm, n, c->obj.row_ptr, c->obj.col,
                           masked ? (const T*)c->g : (const T*)c->obj.val, (const double*)Xc, Y);
      else
        hipLaunchKernelGGL((k_tr_matvec_dense<T>), dim3(ceil_div(n, 32)), dim3(256), 0, sm, n, (int64_t)cfg.ld,
                           Launch<T, 16>::dense_src(c), (const double*)Xc, Y);
      if (r > 0)
        tr_gram<T>(sm, Qm, KB, r, Xc, n, GR, part, P);
      hipLaunchKernelGGL((k_tr_opfix<T>), dim3(ge), dim3(256), 0, sm, Qm, KB, r, (const double*)dcv,
                         (const double*)P, sop, c0, (const double*)Xc, n, Y);
      double* alj = al + (size_t)j * kTrW;
      const double* bprev = j > 0 ? bb + (size_t)(j - 1) * kTrW : nullptr;
      tr_cdot(sm, Xc, Y, n, GR, part, alj);
      hipLaunchKernelGGL(k_tr_three, dim3(ge), dim3(256), 0, sm, (const double*)Y, (const double*)Xc,
                         (const double*)Xp, (const double*)alj, bprev, n, Wn);
      tr_cdot(sm, Wn, Wn, n, GR, part, sm1);
      hipLaunchKernelGGL(k_tr_next, dim3(ge), dim3(256), 0, sm, (const double*)sm1, (const double*)alj, bprev, n,
                         bb + (size_t)j * kTrW, Wn);
      if (hipGetLastError() != hipSuccess) return fail();
      double* old = Xp;
      Xp = Xc;
      Xc = Wn;
      Wn = old;
      done = j + 1;
      if (done % 8 != 0 && done != m) continue;
      if (hipMemcpyAsync(abh.data(), al, (size_t)done * kTrW * 8, hipMemcpyDeviceToHost, sm) != hipSuccess ||
          hipMemcpyAsync(bbh.data(), bb, (size_t)done * kTrW * 8, hipMemcpyDeviceToHost, sm) != hipSuccess ||
          hipStreamSynchronize(sm) != hipSuccess)
        return fail();
      batch_conv = true;
      for (int b = 0; b < nq + np_b; ++b) {
        if (!(nsq[b] > 0.0)) {
          conv[b] = 1;
          continue;
        }
        // T of vector b, truncated at its first vanishing beta (invariant space)
        int len = done;
        bool invariant = false;
        for (int q = 0; q < done; ++q)
          if (bbh[(size_t)q * kTrW + b] == 0.0) {
            len = q + 1;
            invariant = true;
            break;
          }
        std::vector<double> ta(len), tb(std::max(len - 1, 0));
        for (int q = 0; q < len; ++q) ta[q] = abh[(size_t)q * kTrW + b];
        for (int q = 0; q + 1 < len; ++q) tb[q] = bbh[(size_t)q * kTrW + b];
        lq_prev[b] = lq[b];
        lq[b] = std::log(nsq[b]) + log_quad_exp(ta, tb);
        // n steps span the whole space: the quadrature is then exact
        conv[b] = invariant || done >= n || (std::isfinite(lq_prev[b]) && std::fabs(lq[b] - lq_prev[b]) <= tol);
        batch_conv = batch_conv && conv[b];
      }
      if (batch_conv) break;
    }
    all_conv = all_conv && batch_conv;
    max_done = std::max(max_done, done);
    for (int b = 0; b < nq; ++b)
      if (nsq[b] > 0.0) defl.push_back(lq[b]);
    for (int b = nq; b < nq + np_b; ++b)
      tail[next_probe + b - nq] = nsq[b] > 0.0 ? lq[b] : -std::numeric_limits<double>::infinity();
    next_probe += np_b;
  }
  const double ninf = -std::numeric_limits<double>::infinity();
  const double lb_defl = defl.empty() ? ninf : log_sum_exp(defl);
  const double lb_tail = p > 0 ? std::log(weight) + log_sum_exp(tail) : ninf;
  const double lb = log_sum_exp({lb_defl, lb_tail});
  double rel_se = std::numeric_limits<double>::quiet_NaN();
  if (p >= 2) {
    double S = ninf;
    for (double v : tail) S = std::max(S, v);
    if (std::isfinite(S)) {
      double mean = 0.0;
      for (double v : tail) mean += std::exp(v - S);
      mean /= p;
      double var = 0.0;
      for (double v : tail) var += (std::exp(v - S) - mean) * (std::exp(v - S) - mean);
      var /= (p - 1);
      rel_se = var > 0.0 ? std::exp(std::log(weight) + 0.5 * std::log((double)p) + S + 0.5 * std::log(var) - lb) : 0.0;
    } else {
      rel_se = 0.0;
    }
  }
  out->log_b = lb;
  out->log_b_defl = lb_defl;
  out->log_b_tail = lb_tail;
  out->tail_rel_stderr = rel_se;
  out->kd = kd;
  out->steps = max_done;
  out->converged = all_conv ? 1 : 0;
  out->batches = batches;
  return MEG_OK;
}

// barrier error flag set by the step kernel: the grid did not complete a barrier
meg_status check_barrier(meg_ctx c) {
  unsigned err = 0;
  HIPCHK(c, hipMemcpy(&err, c->bar + kBarErr, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (err) return hip_fail(c);
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
  o->cert_resolved = in.cert_resolved;
  o->resid_r1 = in.resid_r1;
  o->cert_L_up = in.cert_L_up;
  o->mu_r1_up = in.mu_r1_up;
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
  meg_status st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
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
  h.polish = 0;
  h.xvalid = 0;
  h.mu_valid = 0;  // the first sweep after a new iterate has no Chebyshev interval yet
  h.cheb_b = 0.0;
  h.pxvalid = 0;  // the shift falls back to the a-priori bound for the new iterate
  h.dxnorm = 0.0;
  h.solve_tol = 0.0;
  std::memset(&h.info, 0, sizeof(Info));
  h.info.t = t - 1;
  HIPCHK(c, hipMemcpyAsync(c->ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, dispatch<DoBasis>(c));
  if (c->da) HIPCHK(c, dispatch<DoDaInit>(c));  // the dual average restarts at log X
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return check_barrier(c);
}

// Sum the elapsed time of the oldest timed launch into the counters.
hipError_t harvest_one(meg_ctx c) {
  const int h = c->ev_head;
  hipError_t e = hipEventSynchronize(c->ev_b[h]);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev_a[h], c->ev_b[h]);
  if (e != hipSuccess) return e;
  c->kernel_ms += ms;
  c->ev_head = (h + 1) % meg_ctx_s::kEvRing;
  --c->ev_count;
  return hipSuccess;
}

// One launch of the step kernel (nsteps iterations) between a HIP event pair.
hipError_t launch_steps(meg_ctx c, int nsteps) {
  if (c->ev_count == meg_ctx_s::kEvRing) {
    const hipError_t e = harvest_one(c);
    if (e != hipSuccess) return e;
  }
  const int slot = (c->ev_head + c->ev_count) % meg_ctx_s::kEvRing;
  hipError_t e = hipEventRecord(c->ev_a[slot], c->stream);
  if (e == hipSuccess) e = dispatch<DoStep>(c, nsteps, false);
  if (e == hipSuccess) e = hipEventRecord(c->ev_b[slot], c->stream);
  if (e != hipSuccess) return e;
  ++c->ev_count;
  ++c->launches;
  return hipSuccess;
}

meg_status check_ctx(meg_ctx c) {
  if (!c) return MEG_ERR_INVALID_ARG;
  if (c->failed) return MEG_ERR_STATE;
  return MEG_OK;
}

meg_status validate(const meg_params* p, const meg_objective* o, const meg_start* s, int* kout) {
  if (!p || !o || !s) return MEG_ERR_INVALID_ARG;
  if (p->n < 2 || p->r < 1 || p->r > p->n - 1) return MEG_ERR_INVALID_ARG;
  if (p->n > 2147483647LL) return MEG_ERR_INVALID_ARG;
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
  if (!(p->inner_tol >= 0.0) || !std::isfinite(p->cert_tol)) return MEG_ERR_INVALID_ARG;
  switch (o->kind) {
    case MEG_GRAD_LINEAR_DENSE:
    case MEG_GRAD_DENOISE_DENSE:
      if (!o->dense || o->ld < p->n) return MEG_ERR_INVALID_ARG;
      if (p->prec == MEG_PREC_F32_BF16X3) {
        // two bf16 planes; rows start on 16-byte boundaries (8-element loads)
        if (!o->dense_lo || o->ld % 8 != 0 || ((uintptr_t)o->dense % 16) != 0 || ((uintptr_t)o->dense_lo % 16) != 0)
          return MEG_ERR_INVALID_ARG;
      }
      break;
    case MEG_GRAD_LINEAR_CSR:
    case MEG_GRAD_MASKED_CSR:
      if (!o->row_ptr || o->nnz < 0 || (o->nnz > 0 && (!o->col || !o->val))) return MEG_ERR_INVALID_ARG;
      if (o->nnz > 2147483647LL) return MEG_ERR_INVALID_ARG;
      if (p->prec == MEG_PREC_F32_BF16X3) return MEG_ERR_UNSUPPORTED;
      break;
    case MEG_GRAD_EXTERNAL:
      if (p->prec == MEG_PREC_F32_BF16X3) return MEG_ERR_UNSUPPORTED;
      break;
    case MEG_GRAD_BILINEAR:
      if (!o->A || !o->b || o->m < 1 || o->lda < p->n || o->batch < 0 || o->batch > 4096) return MEG_ERR_INVALID_ARG;
      if (o->m > (int64_t)1 << 36 || o->lda > (int64_t)1 << 40) return MEG_ERR_INVALID_ARG;
      if (p->prec == MEG_PREC_F32_BF16X3) return MEG_ERR_UNSUPPORTED;
      break;
    case MEG_GRAD_QUADMEAS: {
      if (!o->A || !o->b || !o->batch_idx || o->m < 1 || o->lda < p->n || o->batch_steps < 1) return MEG_ERR_INVALID_ARG;
      if (o->batch < 1 || o->batch > kMaxBatch) return MEG_ERR_INVALID_ARG;
      if (o->m > (int64_t)1 << 40 || o->lda > (int64_t)1 << 40 || o->batch_steps > ((int64_t)1 << 40) / o->batch)
        return MEG_ERR_INVALID_ARG;
      if (p->prec == MEG_PREC_F32_BF16X3) return MEG_ERR_UNSUPPORTED;
      // rows of the pool start on 16-byte boundaries (vector loads)
      const size_t es = (p->prec == MEG_PREC_F64) ? 8 : 4;
      if (((uintptr_t)o->A % 16) != 0 || (o->lda * (int64_t)es) % 16 != 0) return MEG_ERR_INVALID_ARG;
      break;
    }
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
  for (int a = 0; a < s->q; ++a)  // orthonormal start columns
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
  void* bufs[] = {c->Qw,   c->Za,  c->Zb, c->g,  c->quad,    c->ctl,    c->part,     c->gpart,
                  c->sums, c->bar, c->ts, c->lz_prev, c->lz_ws, c->tr_ws, c->bil_G, c->bil_res, c->bil_P,
                  c->da_Y};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  if (c->h_w) (void)hipHostFree(c->h_w);
  for (int i = 0; i < meg_ctx_s::kEvRing; ++i) {
    if (c->ev_a[i]) (void)hipEventDestroy(c->ev_a[i]);
    if (c->ev_b[i]) (void)hipEventDestroy(c->ev_b[i]);
  }
  delete c;
}

// One step with a caller-supplied (or context-formed) gradient G_t: its
// Gershgorin bound, this step's shift and coefficients, one step launch.
meg_status external_step_core(meg_ctx c, const meg_objective* grad, meg_step_info* info) {
  meg_status st = MEG_OK;
  Cfg& cfg = c->cfg;
  const int64_t n = cfg.n;
  if (grad->kind == MEG_GRAD_LINEAR_DENSE) {
    if (!grad->dense || grad->ld < n) return MEG_ERR_INVALID_ARG;
  } else if (grad->kind == MEG_GRAD_LINEAR_CSR) {
    if (!grad->row_ptr || grad->nnz < 0 || grad->nnz > 2147483647LL || (grad->nnz > 0 && (!grad->col || !grad->val)))
      return MEG_ERR_INVALID_ARG;
    // structure check before any kernel reads through the indices
    int h_err = 0;
    int* d_err = (int*)c->sums;
    HIPCHK(c, hipMemsetAsync(d_err, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_check_csr, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0,
                       c->stream, grad->row_ptr, grad->col, n, grad->nnz, d_err);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (h_err) return MEG_ERR_INVALID_ARG;
  } else {
    return MEG_ERR_UNSUPPORTED;
  }
  // this step's operator
  if (grad->kind == MEG_GRAD_LINEAR_DENSE) {
    c->obj.dense = grad->dense;
    c->obj.ld = grad->ld;
    cfg.ld = grad->ld;
    cfg.kind = LINEAR_DENSE;
  } else {
    c->obj.row_ptr = grad->row_ptr;
    c->obj.col = grad->col;
    c->obj.val = grad->val;
    c->obj.nnz = grad->nnz;
    cfg.nnz = grad->nnz;
    cfg.kind = LINEAR_CSR;
  }
  cfg.cache_blocks = 0;  // the pattern may change from step to step
  cfg.cache_nnz = 0;
  // Gershgorin bounds of G_t, then the shift and coefficients of this step
  const int gw = (int)std::max<int64_t>(1, std::min<int64_t>(512, (n + 3) / 4));
  const bool dbl = c->esize == 8;
  if (cfg.kind == LINEAR_DENSE) {
    if (dbl)
      hipLaunchKernelGGL((k_gersh_dense<double>), dim3(gw), dim3(256), 0, c->stream, (const double*)grad->dense, n,
                         grad->ld, c->part);
    else
      hipLaunchKernelGGL((k_gersh_dense<float>), dim3(gw), dim3(256), 0, c->stream, (const float*)grad->dense, n,
                         grad->ld, c->part);
  } else {
    if (dbl)
      hipLaunchKernelGGL((k_gersh_csr<double>), dim3(gw), dim3(256), 0, c->stream, grad->row_ptr, grad->col,
                         (const double*)grad->val, n, c->part);
    else
      hipLaunchKernelGGL((k_gersh_csr<float>), dim3(gw), dim3(256), 0, c->stream, grad->row_ptr, grad->col,
                         (const float*)grad->val, n, c->part);
  }
  hipLaunchKernelGGL(k_external_setup, dim3(1), dim3(64), 0, c->stream, cfg, c->ctl, c->part, gw);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, launch_steps(c, 1));
  // the caller's arrays are read during the call only
  HIPCHK(c, hipStreamSynchronize(c->stream));
  st = sync_ctl(c);
  if (st != MEG_OK) return st;
  if (info) {
    fill_info(*c->h_ctl, info);
    if (!c->bilinear) info->f = __builtin_nan("");  // bilinear: f(X_t) from its residuals
  }
  if (c->h_ctl->status) return (meg_status)c->h_ctl->status;
  if (info && (c->params.flags & MEG_FLAG_STRICT) && !info->converged) return MEG_ERR_NOT_CONVERGED;
  return MEG_OK;
}

// one step of a bilinear-measurement context: residuals, f(X_t) and the dense
// gradient G_t on the device, then the external step with G_t
meg_status bilinear_prepare(meg_ctx c, bool grad) {
  HIPCHK(c, dispatch<DoBilinear>(c, grad));
  if (grad) {
    c->obj.dense = c->bil_G;
    c->obj.ld = c->cfg.n;
    c->cfg.ld = c->cfg.n;
    c->cfg.kind = LINEAR_DENSE;
  }
  return MEG_OK;
}

meg_status bilinear_step(meg_ctx c, meg_step_info* info) {
  meg_status st = bilinear_prepare(c, true);
  if (st != MEG_OK) return st;
  meg_objective g;
  std::memset(&g, 0, sizeof(g));
  g.kind = MEG_GRAD_LINEAR_DENSE;
  g.dense = c->bil_G;
  g.ld = c->cfg.n;
  return external_step_core(c, &g, info);
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
  cfg.rr_from = std::min(2, (int)params->max_inner);
  cfg.eta = params->eta;
  cfg.eps_scale = params->eps_scale;
  cfg.eps_c = params->eps_c;
  cfg.eps_pow = params->eps_pow;
  cfg.inner_tol = params->inner_tol > 0 ? params->inner_tol : (c->esize == 8 ? 1e-10 : 1e-6);
  cfg.unit_round = (c->esize == 8) ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
  cfg.cert_tol = params->cert_tol;
  cfg.xres = (c->esize == 8) ? 1 : 0;  // explicit Ritz residuals in FP64
  cfg.extrap = (c->esize == 4 && !(params->flags & MEG_FLAG_NO_EXTRAPOLATE)) ? 1 : 0;
  cfg.cheb = (params->flags & MEG_FLAG_NO_CHEBYSHEV) ? 0 : 1;
  c->da = (params->flags & MEG_FLAG_DUAL_AVERAGE) != 0;
  if (c->da && ((obj->kind != MEG_GRAD_LINEAR_DENSE && obj->kind != MEG_GRAD_DENOISE_DENSE) ||
                params->prec == MEG_PREC_F32_BF16X3)) {
    delete c;
    return MEG_ERR_UNSUPPORTED;
  }
  if (obj->kind == MEG_GRAD_EXTERNAL || obj->kind == MEG_GRAD_BILINEAR) {
    // the operator family is chosen per step; dense until then (bilinear: always
    // the dense gradient the context forms)
    c->external = true;
    c->bilinear = obj->kind == MEG_GRAD_BILINEAR;
    cfg.kind = LINEAR_DENSE;
    if (c->bilinear) cfg.ld = cfg.n;
  }

  int coop = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) {
    (void)hipGetLastError();
    delete c;
    return MEG_ERR_DEVICE;
  }
  c->device = dev;
  // this device's address of the allocation-free entry point's scratch (once
  // per device, with the device current)
  if (scratch_lookup(dev) != MEG_OK) {
    delete c;
    return MEG_ERR_DEVICE;
  }
  c->P = dispatch<DoGrid>(c);
  if (c->external) {  // a grid that both operator families can launch cooperatively
    cfg.kind = LINEAR_CSR;
    c->P = std::min(c->P, dispatch<DoGrid>(c));
    cfg.kind = LINEAR_DENSE;
  }
  if (c->P < 1) {
    delete c;
    return MEG_ERR_DEVICE;
  }
  c->aux_nwg = std::max(1024, ceil_div(cfg.n, 4));
  // (the dual average's row bounds take n entries)
  const size_t pe = std::max({dispatch<DoPartNeed>(c, c->P), (size_t)c->aux_nwg, (size_t)cfg.n});
  const size_t zbytes = (size_t)cfg.n * k * c->esize;
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 256)) == hipSuccess; };
  bool ok = alloc(&c->Qw, zbytes) && alloc(&c->Za, zbytes) && alloc(&c->Zb, zbytes) &&
            alloc((void**)&c->ctl, sizeof(Ctl)) && alloc((void**)&c->part, pe * 8) &&
            alloc((void**)&c->sums, kPartMax * 8) && alloc((void**)&c->bar, kBarWords * sizeof(unsigned)) &&
            alloc((void**)&c->gpart, (size_t)kBarMaxGroups * kPartMax * 8) &&
            alloc((void**)&c->ts, kTsSlots * sizeof(long long));
  if (ok && obj->kind == MEG_GRAD_MASKED_CSR) ok = alloc(&c->g, (size_t)std::max<int64_t>(obj->nnz, 1) * c->esize);
  if (ok && c->da) ok = alloc(&c->da_Y, (size_t)cfg.n * cfg.n * c->esize);
  if (ok && obj->kind == MEG_GRAD_QUADMEAS) ok = alloc(&c->quad, quad_layout(obj->batch, k, c->esize).bytes);
  if (ok && c->bilinear) {
    // slices of the measurement rows: about 2048 partial-gradient workgroups
    // (eight per compute unit)
    const int64_t tiles = ceil_div(cfg.n, kBilTile), pairs = tiles * (tiles + 1) / 2;
    const int64_t rows = obj->m * std::max(1, (int)obj->batch);
    c->bil_S = (int)std::max<int64_t>(1, std::min<int64_t>({64, 2048 / pairs, ceil_div(rows, 16)}));
    ok = alloc(&c->bil_G, (size_t)cfg.n * cfg.n * c->esize) && alloc((void**)&c->bil_res, (size_t)obj->m * 8) &&
         alloc((void**)&c->bil_P, (size_t)c->bil_S * pairs * kBilTile * kBilTile * 8);
  }
  if (ok) ok = hipHostMalloc((void**)&c->h_ctl, sizeof(Ctl)) == hipSuccess;
  if (ok) ok = hipHostMalloc((void**)&c->h_w, sizeof(meg_ctx_s::HostWords)) == hipSuccess;
  if (ok) std::memset(c->h_w, 0, sizeof(meg_ctx_s::HostWords));
  for (int i = 0; ok && i < meg_ctx_s::kEvRing; ++i)
    ok = hipEventCreate(&c->ev_a[i]) == hipSuccess && hipEventCreate(&c->ev_b[i]) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_ctx(c);
    return MEG_ERR_OUT_OF_MEMORY;
  }
  c->part_elems = pe;
  if (hipMemsetAsync(c->bar, 0, kBarWords * sizeof(unsigned), c->stream) != hipSuccess ||
      hipMemsetAsync(c->ctl, 0, sizeof(Ctl), c->stream) != hipSuccess ||
      hipMemsetAsync(c->ts, 0, kTsSlots * sizeof(long long), c->stream) != hipSuccess) {
    free_ctx(c);
    return MEG_ERR_DEVICE;
  }
  // CSR structure check before any kernel reads through the indices
  if (obj->kind == MEG_GRAD_LINEAR_CSR || obj->kind == MEG_GRAD_MASKED_CSR) {
    int h_err = 0;
    int* d_err = (int*)c->sums;
    if (hipMemsetAsync(d_err, 0, sizeof(int), c->stream) != hipSuccess) {
      free_ctx(c);
      return MEG_ERR_DEVICE;
    }
    hipLaunchKernelGGL(k_check_csr, dim3((unsigned)std::min<int64_t>(1024, (cfg.n + 255) / 256)), dim3(256), 0,
                       c->stream, obj->row_ptr, obj->col, cfg.n, cfg.nnz, d_err);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
      free_ctx(c);
      return MEG_ERR_DEVICE;
    }
    if (h_err) {
      free_ctx(c);
      return MEG_ERR_INVALID_ARG;
    }
    (void)dispatch<DoCache>(c);  // per-workgroup LDS copy of the CSR data, when it fits
  }
  // minibatch index check before any kernel reads the pool through them
  if (obj->kind == MEG_GRAD_QUADMEAS) {
    int h_err = 0;
    int* d_err = (int*)c->sums;
    const int64_t cnt = obj->batch_steps * (int64_t)obj->batch;
    if (hipMemsetAsync(d_err, 0, sizeof(int), c->stream) != hipSuccess) {
      free_ctx(c);
      return MEG_ERR_DEVICE;
    }
    hipLaunchKernelGGL(k_check_idx, dim3((unsigned)std::min<int64_t>(1024, (cnt + 255) / 256)), dim3(256), 0,
                       c->stream, obj->batch_idx, cnt, obj->m, d_err);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
      free_ctx(c);
      return MEG_ERR_DEVICE;
    }
    if (h_err) {
      free_ctx(c);
      return MEG_ERR_INVALID_ARG;
    }
  }
  // data norm (sets ctl->data_norm) and the extreme eigenvalues of the data
  // operator (shift of the subspace iteration); the factored gradient
  // changes every step and bounds its spectrum inside the step instead
  const bool has_data =
      obj->kind != MEG_GRAD_QUADMEAS && obj->kind != MEG_GRAD_EXTERNAL && obj->kind != MEG_GRAD_BILINEAR;
  if (has_data && (dispatch<DoNorm>(c) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)) {
    free_ctx(c);
    return MEG_ERR_DEVICE;
  }
  if (has_data) {
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

// One step of the dual-averaging reading: f(X_t) (when asked), Y <- Y - eta
// grad f(X_t), then the step kernel on the dense operator Y + sigma' I (a
// launch with Y as the context's dense linear operator).
meg_status da_step(meg_ctx c, meg_step_info* info) {
  if (info) HIPCHK(c, dispatch<DoObjective>(c));
  HIPCHK(c, dispatch<DoDaUpdate>(c));
  const void* dsave = c->obj.dense;
  const int64_t ldsave = c->obj.ld;
  const Cfg csave = c->cfg;
  c->obj.dense = c->da_Y;
  c->obj.ld = c->cfg.n;
  c->cfg.kind = LINEAR_DENSE;
  c->cfg.ld = c->cfg.n;
  const hipError_t e = launch_steps(c, 1);
  c->obj.dense = dsave;
  c->obj.ld = ldsave;
  c->cfg = csave;
  HIPCHK(c, e);
  if (!info) return MEG_OK;
  meg_status st = sync_ctl(c);
  if (st != MEG_OK) return st;
  fill_info(*c->h_ctl, info);
  if (c->h_ctl->status) return (meg_status)c->h_ctl->status;
  if ((c->params.flags & MEG_FLAG_STRICT) && !info->converged) return MEG_ERR_NOT_CONVERGED;
  return MEG_OK;
}

meg_status meg_step(meg_ctx c, meg_step_info* info) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (c->bilinear) return bilinear_step(c, info);
  if (c->da) return da_step(c, info);
  if (c->external) return MEG_ERR_INVALID_ARG;
  // f(X_t): the masked objective's gradient phase computes it in the step
  if (info && c->cfg.kind != MASKED_CSR) HIPCHK(c, dispatch<DoObjective>(c));
  HIPCHK(c, launch_steps(c, 1));
  if (!info) return MEG_OK;
  st = sync_ctl(c);
  if (st != MEG_OK) return st;
  fill_info(*c->h_ctl, info);
  if (c->h_ctl->status) return (meg_status)c->h_ctl->status;
  if ((c->params.flags & MEG_FLAG_STRICT) && !info->converged) return MEG_ERR_NOT_CONVERGED;
  return MEG_OK;
}

meg_status meg_step_external(meg_ctx c, const meg_objective* grad, meg_step_info* info) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!c->external || c->bilinear || !grad) return MEG_ERR_INVALID_ARG;
  return external_step_core(c, grad, info);
}

meg_status meg_solve(meg_ctx c, int64_t max_iters, double tol, meg_step_info* last) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (max_iters < 0) return MEG_ERR_INVALID_ARG;
  if (c->bilinear) {  // one step per iteration: each forms its own gradient first
    meg_step_info inf;
    std::memset(&inf, 0, sizeof(inf));
    bool any = false;
    for (int64_t i = 0; i < max_iters; ++i) {
      st = bilinear_step(c, &inf);
      if (st != MEG_OK) return st;
      any = true;
      if (tol > 0.0 && inf.cert_bound <= tol) break;
    }
    if (last) {
      if (any) *last = inf;
      else st = meg_certificate(c, last);
    }
    return st;
  }
  if (c->external) return MEG_ERR_INVALID_ARG;
  if (c->da) {  // one launch per iteration (each updates Y first)
    meg_step_info inf;
    std::memset(&inf, 0, sizeof(inf));
    bool any = false;
    for (int64_t i = 0; i < max_iters; ++i) {
      st = da_step(c, &inf);
      if (st != MEG_OK) return st;
      any = true;
      if (tol > 0.0 && fmax(2.0 * inf.eps_t, inf.cert_L_up) <= tol) break;
    }
    if (last) {
      if (any) *last = inf;
      else st = meg_certificate(c, last);
    }
    return st;
  }
  // Outside this call the device's stop rule is disarmed (solve_tol = 0,
  // stop = 0): only a tolerance arms it, by asynchronous copies from pinned
  // words; the host mirror is refreshed after the launches.
  const bool arm = tol > 0;
  if (arm) {
    c->h_w->tol = tol;
    c->h_w->stop = 0;
    HIPCHK(c, hipMemcpyAsync(&c->ctl->solve_tol, &c->h_w->tol, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(&c->ctl->stop, &c->h_w->stop, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  }
  int64_t done = 0;
  while (done < max_iters) {
    const int m = (int)std::min<int64_t>(kChunkSteps, max_iters - done);
    HIPCHK(c, launch_steps(c, m));
    done += m;
    if (tol > 0 && done < max_iters) {
      st = copy_ctl_to_host(c);
      if (st != MEG_OK) return st;
      if (c->h_ctl->stop || c->h_ctl->status) break;
    }
  }
  st = sync_ctl(c);
  if (st != MEG_OK) return st;
  const int32_t status = c->h_ctl->status;
  if (last) {
    fill_info(*c->h_ctl, last);
    last->f = __builtin_nan("");
  }
  if (arm) {  // disarm: ordered before any later work on the stream, no wait here
    c->h_ctl->solve_tol = 0.0;
    c->h_ctl->stop = 0;
    HIPCHK(c, hipMemcpyAsync(&c->ctl->solve_tol, &c->h_w->zero_d, sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(&c->ctl->stop, &c->h_w->zero_i, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  }
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
  if (c->external && !c->bilinear) return MEG_ERR_UNSUPPORTED;  // f is the caller's
  if (!f) return MEG_ERR_INVALID_ARG;
  if (c->bilinear) {
    st = bilinear_prepare(c, false);
    if (st != MEG_OK) return st;
  } else {
    HIPCHK(c, dispatch<DoObjective>(c));
  }
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
  if (V) {  // V = (B Wb)[:, :r], B = block src
    const int k = cfg.k;
    const size_t cnt = (size_t)cfg.n * k;
    std::vector<double> B(cnt);
    const void* blk = block(c, c->h_ctl->src);
    if (c->esize == 8) {
      HIPCHK(c, hipMemcpy(B.data(), blk, cnt * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> Bf(cnt);
      HIPCHK(c, hipMemcpy(Bf.data(), blk, cnt * 4, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < cnt; ++i) B[i] = Bf[i];
    }
    const double* Wb = c->h_ctl->Wb;
    for (int64_t i = 0; i < cfg.n; ++i)
      for (int l = 0; l < cfg.r; ++l) {
        double v = 0.0;
        for (int q = 0; q < k; ++q) v += B[(size_t)i * k + q] * Wb[q * k + l];
        V[(size_t)l * cfg.n + i] = v;
      }
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
  HIPCHK(c, hipMemcpy(p + 32 + sizeof(Ctl), block(c, c->h_ctl->src), qbytes, hipMemcpyDeviceToHost));
  *bytes = need;
  return MEG_OK;
}

meg_status meg_set_state(meg_ctx c, const void* buf, size_t bytes) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (c->da) return MEG_ERR_UNSUPPORTED;  // the dual average Y is not part of the state blob
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
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  const int64_t iters = c->h_ctl->iters_done, applies = c->h_ctl->applies_done, jac = c->h_ctl->jacobi_done;
  std::memcpy(c->h_ctl, p + 32, sizeof(Ctl));
  c->h_ctl->iters_done = iters;  // work counters describe this context, not the blob
  c->h_ctl->applies_done = applies;
  c->h_ctl->jacobi_done = jac;
  HIPCHK(c, hipMemcpyAsync(c->ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  if (c->h_ctl->src < 0 || c->h_ctl->src > 2) return MEG_ERR_STATE;
  HIPCHK(c, hipMemcpyAsync(block(c, c->h_ctl->src), p + 32 + sizeof(Ctl), qbytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MEG_OK;
}

meg_status meg_profile_step(meg_ctx c, meg_kernel_times* out) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (c->da) return MEG_ERR_UNSUPPORTED;
  if (!out || c->external) return MEG_ERR_INVALID_ARG;  // an external G_t is borrowed for one call only
  std::memset(out, 0, sizeof(*out));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(c);
  }
  bool ok = hipMemsetAsync(c->ts, 0, kTsSlots * sizeof(long long), c->stream) == hipSuccess &&
            hipEventRecord(e0, c->stream) == hipSuccess && dispatch<DoStep>(c, 1, true) == hipSuccess &&
            hipEventRecord(e1, c->stream) == hipSuccess && hipStreamSynchronize(c->stream) == hipSuccess;
  float ms = 0.f;
  if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return hip_fail(c);
  c->kernel_ms += ms;
  ++c->launches;
  std::vector<long long> ts(kTsSlots);
  HIPCHK(c, hipMemcpy(ts.data(), c->ts, kTsSlots * sizeof(long long), hipMemcpyDeviceToHost));
  st = sync_ctl(c);
  if (st != MEG_OK) return st;
  int dev = 0, khz = 100000;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  const double tick_ms = 1.0 / (double)std::max(khz, 1);
  const int mi = c->cfg.max_inner;
  const int used = std::max(1, std::min(mi, (int)c->h_ctl->info.inner_iters));
  out->kernel_ms = ms;
  out->prep_ms = (ts[1] - ts[0]) * tick_ms;
  for (int s = 1; s <= used; ++s) {
    out->apply_ms[s - 1] = (ts[2 * s] - ts[2 * s - 1]) * tick_ms;
    out->small_ms[s - 1] = (ts[2 * s + 1] - ts[2 * s]) * tick_ms;
  }
  out->finalize_ms = 0.0;  // the step ends inside its last sweep's small solve
  out->sweeps_active = used;
  out->workgroups = c->P;
  const int P = c->P;
  for (int s = 1; s <= std::min(used, kTsWgSweeps); ++s) {
    const long long* st = &ts[kTsWg + (size_t)(2 * (s - 1)) * P];
    const long long* ar = &ts[kTsWg + (size_t)(2 * (s - 1) + 1) * P];
    long long dmin = LLONG_MAX, dmax = 0, smin = LLONG_MAX, smax = 0, amax = 0;
    double dsum = 0.0;
    for (int w = 0; w < P; ++w) {
      const long long d = ar[w] - st[w];
      dmin = std::min(dmin, d);
      dmax = std::max(dmax, d);
      dsum += (double)d;
      smin = std::min(smin, st[w]);
      smax = std::max(smax, st[w]);
      amax = std::max(amax, ar[w]);
    }
    out->wg_apply_ms[s - 1][0] = dmin * tick_ms;
    out->wg_apply_ms[s - 1][1] = dsum / P * tick_ms;
    out->wg_apply_ms[s - 1][2] = dmax * tick_ms;
    out->wg_skew_ms[s - 1] = (smax - smin) * tick_ms;
    out->reduce_ms[s - 1] = (ts[2 * s] - amax) * tick_ms;
  }
  const int rs = c->cfg.rr_from;
  if (used >= rs && ts[kTsRR + 3] > 0) {
    out->rr_ms[0] = (ts[kTsRR] - ts[2 * rs]) * tick_ms;
    out->rr_ms[1] = (ts[kTsRR + 1] - ts[kTsRR]) * tick_ms;
    out->rr_ms[2] = (ts[kTsRR + 2] - ts[kTsRR + 1]) * tick_ms;
    out->rr_tail_ms = (ts[kTsRR + 3] - ts[kTsRR + 2]) * tick_ms;
    out->jacobi_sweeps = (int32_t)ts[kTsRR + 4];
  }
  return c->h_ctl->status ? (meg_status)c->h_ctl->status : MEG_OK;
}

// The gradient at the current iterate made available to the Lanczos runs
// (bilinear: formed; masked: its values on the pattern) together with
// <X_t, G> and the materialised basis; the control block copied to the host.
meg_status prepare_gradient(meg_ctx c, double* x_dot_g) {
  meg_status st = MEG_OK;
  if (c->bilinear) {  // G at the current iterate, as the linear operator of the run
    st = bilinear_prepare(c, true);
    if (st != MEG_OK) return st;
  }
  HIPCHK(c, dispatch<DoXdotG>(c));
  const int nwg = ceil_div(c->cfg.n, 4);
  std::vector<double> part(nwg);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(part.data(), c->part, nwg * sizeof(double), hipMemcpyDeviceToHost));
  double xg = 0.0;
  for (int w = 0; w < nwg; ++w) xg += part[w];
  if (x_dot_g) *x_dot_g = xg;
  return copy_ctl_to_host(c);
}

meg_status dual_gap_with(meg_ctx c, int32_t max_steps, double tol, const LzWs& ws, bool warm, meg_dual_gap_info* out) {
  double xg = 0.0;
  meg_status st = prepare_gradient(c, &xg);
  if (st != MEG_OK) return st;
  st = (c->esize == 8) ? lanczos_grad_min<double>(c, max_steps, tol, ws, 0, warm, out)
                       : lanczos_grad_min<float>(c, max_steps, tol, ws, 0, warm, out);
  if (st != MEG_OK) return st;
  out->x_dot_g = xg;
  out->gap = xg - out->lambda_min;
  out->t = c->h_ctl->t;
  return MEG_OK;
}

meg_status dual_gap_args(meg_ctx c, int32_t max_steps, double tol, meg_dual_gap_info* out) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!out || max_steps < 1 || !(tol >= 0.0)) return MEG_ERR_INVALID_ARG;
  if ((c->external && !c->bilinear) || c->cfg.kind == QUADMEAS) return MEG_ERR_UNSUPPORTED;
  std::memset(out, 0, sizeof(*out));
  return MEG_OK;
}

meg_status meg_dual_gap(meg_ctx c, int32_t max_steps, double tol, meg_dual_gap_info* out) {
  meg_status st = dual_gap_args(c, max_steps, tol, out);
  if (st != MEG_OK) return st;
  LzWs ws;
  st = ctx_lz_ws(c, lz_steps(c->cfg.n, 0, max_steps), &ws);
  if (st != MEG_OK) return st;
  return dual_gap_with(c, max_steps, tol, ws, true, out);
}

meg_status meg_dual_gap_static(meg_ctx c, int32_t max_steps, double tol, meg_dual_gap_info* out) {
  meg_status st = dual_gap_args(c, max_steps, tol, out);
  if (st != MEG_OK) return st;
  const int m = lz_steps(c->cfg.n, 0, max_steps);
  if (lz_ws_need(c->cfg.n, m) > kStaticScratchDoubles) return MEG_ERR_INVALID_ARG;
  double* base = nullptr;
  st = static_scratch(c, &base);
  if (st != MEG_OK) return st;
  return dual_gap_with(c, max_steps, tol, lz_ws_carve(base, c->cfg.n, m), false, out);
}

meg_status meg_certificate_bound(meg_ctx c, int32_t max_steps, double tol, meg_cert_bound_info* out) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (c->da) return MEG_ERR_UNSUPPORTED;  // its matrix is Y, not log X_t - eta G
  if (!out || max_steps < 1 || !(tol >= 0.0)) return MEG_ERR_INVALID_ARG;
  if ((c->external && !c->bilinear) || c->cfg.kind == QUADMEAS) return MEG_ERR_UNSUPPORTED;
  std::memset(out, 0, sizeof(*out));
  const int r = c->cfg.r;
  if (c->cfg.n - r < 1) return MEG_ERR_INVALID_ARG;
  LzWs ws;
  st = ctx_lz_ws(c, lz_steps(c->cfg.n, r, max_steps), &ws);
  if (st != MEG_OK) return st;
  st = prepare_gradient(c, nullptr);
  if (st != MEG_OK) return st;
  meg_dual_gap_info g{};
  st = (c->esize == 8) ? lanczos_grad_min<double>(c, max_steps, tol, ws, r, false, &g)
                       : lanczos_grad_min<float>(c, max_steps, tol, ws, r, false, &g);
  if (st != MEG_OK) return st;
  // lambda_{r+1}(M_t) <= log alpha_t - eta lambda_min(G on V_t's complement),
  // with the Ritz value lowered by its residual
  const Ctl& h = *c->h_ctl;
  out->lambda_min_defl = g.lambda_min;
  out->resid = g.resid;
  out->steps = g.steps;
  out->converged = g.converged;
  out->t = h.t;
  out->mu_up = std::log(h.alpha) - c->cfg.eta * (g.lambda_min - g.resid);
  // arm the next step (iteration t): its certificate may use the bound
  HIPCHK(c, hipMemcpyAsync(&c->ctl->mu_up, &out->mu_up, sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(&c->ctl->mu_up_t, &out->t, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MEG_OK;
}

meg_status meg_trace_exp(meg_ctx c, const double* probes, int32_t p, double weight, int32_t max_steps, double tol,
                         meg_trace_info* out) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (c->da) return MEG_ERR_UNSUPPORTED;
  if (!out || p < 0 || (p > 0 && !probes) || !(weight > 0.0) || max_steps < 1 || !(tol >= 0.0))
    return MEG_ERR_INVALID_ARG;
  if ((c->external && !c->bilinear) || c->cfg.kind == QUADMEAS) return MEG_ERR_UNSUPPORTED;
  std::memset(out, 0, sizeof(*out));
  if (c->bilinear) {  // G at the current iterate: M_t = log X_t - eta G as for a linear objective
    st = bilinear_prepare(c, true);
    if (st != MEG_OK) return st;
  }
  HIPCHK(c, dispatch<DoXdotG>(c));  // materialises the basis; masked: the gradient values
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  st = (c->esize == 8) ? trace_exp_run<double>(c, probes, p, weight, max_steps, tol, out)
                       : trace_exp_run<float>(c, probes, p, weight, max_steps, tol, out);
  if (st != MEG_OK) return st;
  out->t = c->h_ctl->t;
  return MEG_OK;
}

meg_status meg_certificate_full(meg_ctx c, const meg_trace_info* tr, double* cert_L_full, int32_t* holds) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!tr || !cert_L_full || !holds) return MEG_ERR_INVALID_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  const Info& in = c->h_ctl->info;
  if (in.t != tr->t || !(in.eps_t > 0.0)) return MEG_ERR_INVALID_ARG;
  const double L = std::log((double)(c->cfg.n - c->cfg.r)) + in.mu_r1 - std::log(in.eps_t) - tr->log_b;
  *cert_L_full = L;
  // mu_{r+1} is the step's Ritz value, a lower bound: a claim uses the
  // step's upper bound of it (L_full moves one for one with mu_{r+1})
  const double L_up = L + (in.mu_r1_up - in.mu_r1);
  *holds = (std::isfinite(L_up) && L_up <= 2.0 * in.eps_t) ? 1 : 0;
  return MEG_OK;
}

meg_status meg_solve_to_gap(meg_ctx c, int64_t max_iters, double tol, int32_t check_every, meg_step_info* last,
                            meg_dual_gap_info* gap) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (c->da) return MEG_ERR_UNSUPPORTED;
  if (max_iters < 0 || !(tol > 0.0) || check_every < 1 || check_every > kChunkSteps) return MEG_ERR_INVALID_ARG;
  if (c->external || c->cfg.kind == QUADMEAS) return MEG_ERR_UNSUPPORTED;
  meg_dual_gap_info g{};
  st = meg_dual_gap(c, 256, 1e-8, &g);
  int64_t done = 0;
  while (st == MEG_OK && done < max_iters && g.gap > tol) {
    const int m = (int)std::min<int64_t>(check_every, max_iters - done);
    HIPCHK(c, launch_steps(c, m));
    done += m;
    st = sync_ctl(c);
    if (st != MEG_OK) return st;
    if (c->h_ctl->status) return (meg_status)c->h_ctl->status;
    st = meg_dual_gap(c, 256, 1e-8, &g);
  }
  if (st != MEG_OK) return st;
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  if (last) {
    fill_info(*c->h_ctl, last);
    last->f = __builtin_nan("");
  }
  if (gap) *gap = g;
  return MEG_OK;
}

meg_status meg_get_counters(meg_ctx c, meg_counters* out, int32_t reset) {
  meg_status st = check_ctx(c);
  if (st != MEG_OK) return st;
  if (!out) return MEG_ERR_INVALID_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  while (c->ev_count > 0) HIPCHK(c, harvest_one(c));
  st = copy_ctl_to_host(c);
  if (st != MEG_OK) return st;
  std::memset(out, 0, sizeof(*out));
  out->launches = c->launches;
  out->iterations = c->h_ctl->iters_done - c->base_iters;
  out->applies = c->h_ctl->applies_done - c->base_applies;
  out->workgroups = c->P;
  out->jacobi_sweeps = (int32_t)std::min<int64_t>(c->h_ctl->jacobi_done - c->base_jacobi, INT32_MAX);
  out->kernel_ms = c->kernel_ms;
  out->extrapolated = c->h_ctl->extrap_done - c->base_extrap;
  out->unconverged = c->h_ctl->unconv_done - c->base_unconv;
  if (reset) {
    c->launches = 0;
    c->kernel_ms = 0.0;
    c->base_iters = c->h_ctl->iters_done;
    c->base_applies = c->h_ctl->applies_done;
    c->base_jacobi = c->h_ctl->jacobi_done;
    c->base_extrap = c->h_ctl->extrap_done;
    c->base_unconv = c->h_ctl->unconv_done;
  }
  return MEG_OK;
}

void meg_destroy(meg_ctx c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_ctx(c);
}

}  // extern "C"
