// Batched server of the low-rank MEG library: the meg_server_* entry points
// declared in include/meg.h.
//
// Many independent instances (dense denoising or linear objective, bf16
// planes, FP32 state, k = 16) are resident at once.  Each launch of the
// batched step kernel k_serve runs every resident instance on its own team
// of workgroups for up to launch_steps iterations; between launches the
// host retires finished instances and admits queued requests (arrival
// order) as workgroups and arena memory free up.  Per instance the device
// holds, in one arena block: the control block, three n x k blocks, the
// two bf16 planes of M (split once at admission), and the team's partials,
// reduction buffers and barrier words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/meg.h"
#include "meg_host.hpp"
#include "meg_kernels.hpp"

using namespace meg;

namespace {

constexpr int kNT = 512;
constexpr int kKB = 16;
constexpr int kMaxSlots = 256;
constexpr int kProbeSlot = kMaxSlots;  // slot index used by the autotuner
constexpr int kGershWg = 256;          // workgroups of the Gershgorin pass
constexpr double kWallClockHz = 1.0e8; // device wall clock (wall_clock64) of gfx950
using Shape = StepShape<float, kKB, OP_DENSE_X3, kNT>;
using SMem = ApplySmem<float, kKB, Shape::ROWS, Shape::GWROWS>;

const void* serve_kernel() { return reinterpret_cast<const void*>(&k_serve<float, kKB, OP_DENSE_X3, kNT>); }
const void* basis_kernel() { return reinterpret_cast<const void*>(&k_basis<float, kKB, OP_DENSE_X3, kNT>); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t plane_ld(int64_t n) { return (n + 7) & ~(int64_t)7; }

// byte offsets of one instance's block in the arena
struct Layout {
  size_t ctl, z0, z1, z2, hi, lo, part, gpart, sums, bar, bytes;
};
Layout layout(int64_t n, int nwg) {
  Layout L;
  size_t o = 0;
  const size_t zb = (size_t)n * kKB * sizeof(float);
  const size_t pb = (size_t)n * plane_ld(n) * 2;
  const size_t pst = SMem::PSTRIDE;
  const int ng = (nwg + kBarGroupSize - 1) / kBarGroupSize;
  L.ctl = o;   o = align256(o + sizeof(Ctl));
  L.z0 = o;    o = align256(o + zb);
  L.z1 = o;    o = align256(o + zb);
  L.z2 = o;    o = align256(o + zb);
  L.hi = o;    o = align256(o + pb);
  L.lo = o;    o = align256(o + pb);
  L.part = o;  o = align256(o + std::max<size_t>((size_t)nwg * pst, 2 * kGershWg) * sizeof(double));
  L.gpart = o; o = align256(o + (size_t)ng * pst * sizeof(double));
  L.sums = o;  o = align256(o + pst * sizeof(double));
  L.bar = o;   o = align256(o + kBarWords * sizeof(unsigned));
  L.bytes = o;
  return L;
}

// first-fit allocator over the device arena (host bookkeeping; blocks are
// 256-byte aligned and coalesced on release)
struct Arena {
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  void init(size_t s) {
    size = s;
    used = peak = 0;
    free_.clear();
    free_[0] = s;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, o2 = it->first + bytes;
      free_.erase(it);
      if (rest) free_[o2] = rest;
      used += bytes;
      peak = std::max(peak, used);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// autotuned team sizes for one n, and the measured time per step (3 sweeps)
// of every timed team size
struct Tuned {
  int lat = 1, thr = 1;
  std::map<int, double> ms_per_step;
  double step_ms(int P) const {  // nearest timed size, scaled by the team ratio
    if (ms_per_step.empty()) return 1.0;
    auto it = ms_per_step.lower_bound(P);
    if (it == ms_per_step.end()) --it;
    return it->second * (double)it->first / (double)P;
  }
};

struct Req {
  meg_request r{};
  std::vector<double> V0, lam0;
  int state = 0, status = MEG_OK;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int slot = -1, nwg = 0;
  size_t off = 0, bytes = 0;
  int64_t iters = 0, applies = 0;
  double step_ms = 1.0;  // autotuner's time per step at its team size (relative speed)
  meg_step_info last{};
  std::vector<double> V, d;
  double alpha = 0;
};

}  // namespace

struct meg_server_s {
  meg_server_params p{};
  hipStream_t stream = nullptr;
  char* arena_base = nullptr;
  Arena arena;
  Slot<float>* d_slots = nullptr;
  Slot<float>* h_slots = nullptr;  // pinned
  int2* d_team = nullptr;
  int2* h_team = nullptr;          // pinned
  SlotSummary* d_sum = nullptr;
  SlotSummary* h_sum = nullptr;    // pinned
  ServeParams* d_prm = nullptr;
  ServeParams* h_prm = nullptr;    // pinned
  // graph mode: the per-round sequence (table copies, the batched kernel on
  // the whole capacity, the summary, its read-back) captured once, replayed
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_coop = false;         // the captured kernel node is a cooperative launch
  int capacity = 0;                // co-resident workgroups of k_serve
  int free_wg = 0;
  std::vector<int64_t> slot_req;   // request resident in each slot, or -1
  std::map<int64_t, Req> reqs;
  std::deque<int64_t> queue;
  std::map<int64_t, Tuned> team;  // autotuned team sizes per n
  int64_t next_id = 1;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  int64_t launch_seq = 0;
  double last_launch_ms = 0.0;
  int64_t submitted = 0, completed = 0, failed_reqs = 0, launches = 0, iterations = 0;
  double kernel_ms = 0;
  std::chrono::steady_clock::time_point t0;
  bool failed = false;
};

namespace {

double now_ms(meg_server s) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s->t0).count();
}

meg_status fail(meg_server s) {
  s->failed = true;
  (void)hipGetLastError();
  return MEG_ERR_DEVICE;
}

#define SCHK(s, x)                            \
  do {                                        \
    if ((x) != hipSuccess) return fail(s);    \
  } while (0)

meg_status validate_request(const meg_request* q) {
  if (!q) return MEG_ERR_INVALID_ARG;
  if (q->kind != MEG_GRAD_DENOISE_DENSE && q->kind != MEG_GRAD_LINEAR_DENSE) return MEG_ERR_UNSUPPORTED;
  if (q->n < 16 || q->n > 32768 || q->r < 1 || q->r > q->n - 1 || q->oversample < 0) return MEG_ERR_INVALID_ARG;
  const int k = meg_block_size(q->r, q->oversample);
  if (k == 0) return MEG_ERR_INVALID_ARG;
  if (k != kKB) return MEG_ERR_UNSUPPORTED;
  if (!q->M || q->ld < q->n) return MEG_ERR_INVALID_ARG;
  if (q->max_iters < 1 || q->max_inner < 1 || q->max_inner > 64) return MEG_ERR_INVALID_ARG;
  if (!(q->eta > 0.0) || !std::isfinite(q->eta)) return MEG_ERR_INVALID_ARG;
  if (!(q->eps_scale > 0.0) || !std::isfinite(q->eps_c) || !(q->eps_pow >= 0.0) || q->eps_c + 1.0 <= 0.0)
    return MEG_ERR_INVALID_ARG;
  const double eps0 = q->eps_scale / std::pow(q->eps_c + 1.0, q->eps_pow);
  if (!(eps0 > 0.0 && eps0 <= 0.75)) return MEG_ERR_INVALID_ARG;
  if (q->q < 1 || q->q > q->r || !q->V0 || !q->lambda0) return MEG_ERR_INVALID_ARG;
  double sum = 0.0;
  for (int i = 0; i < q->q; ++i) {
    if (!(q->lambda0[i] >= 0.0)) return MEG_ERR_INVALID_ARG;
    sum += q->lambda0[i];
  }
  if (std::fabs(sum - 1.0) > 1e-8) return MEG_ERR_INVALID_ARG;
  for (int a = 0; a < q->q; ++a)
    for (int b = a; b < q->q; ++b) {
      double dot = 0.0;
      for (int64_t i = 0; i < q->n; ++i) dot += q->V0[(size_t)a * q->n + i] * q->V0[(size_t)b * q->n + i];
      if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-6) return MEG_ERR_INVALID_ARG;
    }
  return MEG_OK;
}

// largest useful team for n: one 64-row block per workgroup at most
int max_team(meg_server s, int64_t n) {
  const int blocks = (int)((n + Shape::ROWS - 1) / Shape::ROWS);
  return std::max(1, std::min({blocks, s->capacity, kBarGroupSize * kBarMaxGroups}));
}

// Set up an instance in its arena block (queued on the server stream):
// control block, bf16 planes, Gershgorin bounds, start basis and its
// orthonormalising transform.  Fills the slot record (nsteps = 0).
meg_status setup_instance(meg_server s, const meg_request& q, const double* V0, const double* lam0, int nwg,
                          char* base, const Layout& L, int min_inner, int max_inner, Slot<float>* slot) {
  const int64_t n = q.n, ld = plane_ld(n);
  Ctl* ctl = (Ctl*)(base + L.ctl);
  float* Z[3] = {(float*)(base + L.z0), (float*)(base + L.z1), (float*)(base + L.z2)};
  uint16_t* hi = (uint16_t*)(base + L.hi);
  uint16_t* lo = (uint16_t*)(base + L.lo);
  Bufs b{(double*)(base + L.part), (double*)(base + L.gpart), (double*)(base + L.sums), (unsigned*)(base + L.bar),
         nullptr};
  if (nwg == 1) b.sums = b.part;  // a one-workgroup team reads its own partials
  Cfg cfg{};
  cfg.n = n;
  cfg.ld = ld;
  cfg.r = q.r;
  cfg.k = kKB;
  cfg.kind = q.kind;
  cfg.prec = MEG_PREC_F32_BF16X3;
  cfg.min_inner = min_inner;
  cfg.max_inner = max_inner;
  cfg.rr_from = std::min(2, max_inner);
  cfg.eta = q.eta;
  cfg.eps_scale = q.eps_scale;
  cfg.eps_c = q.eps_c;
  cfg.eps_pow = q.eps_pow;
  cfg.inner_tol = 1e-6;
  cfg.unit_round = 5.9604644775390625e-08;
  cfg.cert_tol = 0.0;  // resolve the (r+1)-th pair when the stop rule could act on it
  cfg.extrap = 1;
  cfg.cheb = 1;
  // control block: X_1 = (1 - eps_0) X_0 + (eps_0 / n) I (Algorithm 2, initialisation)
  Ctl h;
  std::memset(&h, 0, sizeof(h));
  const double eps0 = q.eps_scale / std::pow(q.eps_c + 1.0, q.eps_pow);
  h.alpha = eps0 / (double)n;
  for (int l = 0; l < KMAX; ++l) {
    const double dl = (l < q.q) ? (1.0 - eps0) * lam0[l] : 0.0;
    h.d[l] = (l < q.r) ? dl : 0.0;
    h.c[l] = (l < q.r) ? std::log(h.alpha + h.d[l]) - std::log(h.alpha) : 0.0;
  }
  h.t = 1;
  h.sweep = 1;
  h.src = 0;
  h.solve_tol = q.tol > 0 ? q.tol : 0.0;
  h.info.t = 0;
  SCHK(s, hipMemcpyAsync(ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, s->stream));
  SCHK(s, hipMemsetAsync(b.bar, 0, kBarWords * sizeof(unsigned), s->stream));
  const int64_t cnt = n * ld;
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)std::min<int64_t>(4096, (cnt + 255) / 256)), dim3(256), 0,
                     s->stream, q.M, q.ld, n, hi, lo, ld);
  const int gw = (int)std::min<int64_t>(kGershWg, (n + 3) / 4);
  hipLaunchKernelGGL(k_gersh, dim3(gw), dim3(256), 0, s->stream, hi, lo, n, ld, b.part);
  hipLaunchKernelGGL(k_gersh_finish, dim3(1), dim3(64), 0, s->stream, ctl, b.part, gw);
  SCHK(s, hipGetLastError());
  std::vector<double> B;
  if (!build_basis(n, kKB, q.q, V0, q.seed + 7919u, B)) return MEG_ERR_INVALID_ARG;
  std::vector<float> Bf(B.size());
  for (size_t i = 0; i < B.size(); ++i) Bf[i] = (float)B[i];
  // synchronous copy: the host vectors go out of scope here
  SCHK(s, hipStreamSynchronize(s->stream));
  SCHK(s, hipMemcpy(Z[0], Bf.data(), Bf.size() * sizeof(float), hipMemcpyHostToDevice));
  void* args[] = {&cfg, &ctl, &Z[0], &Z[1], &Z[2], &b};
  SCHK(s, hipLaunchCooperativeKernel(basis_kernel(), dim3(nwg), dim3(kNT), args, 0, s->stream));
  Data<float> dat{};
  dat.Dhi = hi;
  dat.Dlo = lo;
  *slot = Slot<float>{cfg, ctl, dat, Z[0], Z[1], Z[2], b, nwg, 0};
  return MEG_OK;
}

// Capture the per-round sequence once: slot table, team table (whole
// capacity) and launch parameters copied from their pinned host mirrors,
// the batched kernel over the whole capacity (workgroups without a team
// exit at once), the summary kernel and its read-back.  The kernel node is
// a cooperative launch when the runtime captures one, else an ordinary
// launch of no more workgroups than are co-resident.
meg_status capture_graph(meg_server s) {
  for (int attempt = 0; attempt < 2 && !s->graph_exec; ++attempt) {
    const bool coop = attempt == 0;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(s);
    bool ok = hipMemcpyAsync(s->d_slots, s->h_slots, sizeof(Slot<float>) * (kMaxSlots + 1), hipMemcpyHostToDevice,
                             s->stream) == hipSuccess &&
              hipMemcpyAsync(s->d_team, s->h_team, sizeof(int2) * s->capacity, hipMemcpyHostToDevice, s->stream) ==
                  hipSuccess &&
              hipMemcpyAsync(s->d_prm, s->h_prm, sizeof(ServeParams), hipMemcpyHostToDevice, s->stream) ==
                  hipSuccess;
    if (ok) {
      void* args[] = {&s->d_slots, &s->d_team, &s->d_prm};
      if (coop) {
        ok = hipLaunchCooperativeKernel(serve_kernel(), dim3(s->capacity), dim3(kNT), args, 0, s->stream) ==
             hipSuccess;
      } else {
        hipLaunchKernelGGL((k_serve<float, kKB, OP_DENSE_X3, kNT>), dim3(s->capacity), dim3(kNT), 0, s->stream,
                           s->d_slots, s->d_team, s->d_prm);
        ok = hipGetLastError() == hipSuccess;
      }
    }
    if (ok) {
      hipLaunchKernelGGL((k_serve_summary<float>), dim3((kMaxSlots + 1 + 255) / 256), dim3(256), 0, s->stream,
                         s->d_slots, kMaxSlots + 1, s->d_sum);
      ok = hipGetLastError() == hipSuccess &&
           hipMemcpyAsync(s->h_sum, s->d_sum, sizeof(SlotSummary) * (kMaxSlots + 1), hipMemcpyDeviceToHost,
                          s->stream) == hipSuccess;
    }
    const bool ended = hipStreamEndCapture(s->stream, &g) == hipSuccess;
    (void)hipGetLastError();
    if (ok && ended && g && hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0) == hipSuccess) {
      s->graph = g;
      s->graph_coop = coop;
    } else {
      if (g) (void)hipGraphDestroy(g);
      s->graph_exec = nullptr;
      (void)hipGetLastError();
    }
  }
  return s->graph_exec ? MEG_OK : fail(s);
}

// one launch of the batched kernel over the slots listed, at most `steps`
// each, within a time budget (ms, <= 0: none); returns the HIP-event time in ms
meg_status launch_serve(meg_server s, const std::vector<int>& slots, const std::vector<int>& steps, double* ms,
                        double budget_ms = 0.0) {
  int w = 0;
  for (size_t i = 0; i < slots.size(); ++i) {
    Slot<float>& sl = s->h_slots[slots[i]];
    sl.nsteps = steps[i];
    for (int k = 0; k < sl.nwg; ++k) s->h_team[w++] = make_int2(slots[i], k);
  }
  if (w == 0) return MEG_OK;
  s->h_prm->seq = ++s->launch_seq;
  s->h_prm->budget = budget_ms > 0.0 ? (long long)(budget_ms * 1e-3 * kWallClockHz) : 0;
  if (s->p.flags & MEG_SERVER_FLAG_GRAPH) {
    for (int k = w; k < s->capacity; ++k) s->h_team[k] = make_int2(-1, 0);  // idle workgroups exit
    if (!s->graph_exec) {
      meg_status st = capture_graph(s);
      if (st != MEG_OK) return st;
    }
    SCHK(s, hipEventRecord(s->ev_a, s->stream));
    SCHK(s, hipGraphLaunch(s->graph_exec, s->stream));
    SCHK(s, hipEventRecord(s->ev_b, s->stream));
  } else {
    SCHK(s, hipMemcpyAsync(s->d_slots, s->h_slots, sizeof(Slot<float>) * (kMaxSlots + 1), hipMemcpyHostToDevice,
                           s->stream));
    SCHK(s, hipMemcpyAsync(s->d_team, s->h_team, sizeof(int2) * w, hipMemcpyHostToDevice, s->stream));
    SCHK(s, hipMemcpyAsync(s->d_prm, s->h_prm, sizeof(ServeParams), hipMemcpyHostToDevice, s->stream));
    SCHK(s, hipEventRecord(s->ev_a, s->stream));
    void* args[] = {&s->d_slots, &s->d_team, &s->d_prm};
    SCHK(s, hipLaunchCooperativeKernel(serve_kernel(), dim3(w), dim3(kNT), args, 0, s->stream));
    SCHK(s, hipEventRecord(s->ev_b, s->stream));
    hipLaunchKernelGGL((k_serve_summary<float>), dim3((kMaxSlots + 1 + 255) / 256), dim3(256), 0, s->stream,
                       s->d_slots, kMaxSlots + 1, s->d_sum);
    SCHK(s, hipGetLastError());
    SCHK(s, hipMemcpyAsync(s->h_sum, s->d_sum, sizeof(SlotSummary) * (kMaxSlots + 1), hipMemcpyDeviceToHost,
                           s->stream));
  }
  SCHK(s, hipStreamSynchronize(s->stream));
  float e = 0.f;
  SCHK(s, hipEventElapsedTime(&e, s->ev_a, s->ev_b));
  *ms = e;
  return MEG_OK;
}

// Team sizes for n: time the batched kernel on a synthetic instance of that
// n (a spiked denoising matrix, fixed 3 sweeps per step) for every
// candidate team size P (powers of two up to one 64-row block per
// workgroup).  Latency choice: the smallest P within 15 % of the fastest;
// throughput choice: the least workgroup time P t(P) per iteration.
meg_status tune(meg_server s, int64_t n, int* lat, int* thr) {
  if (s->p.fixed_team > 0) {  // set by the caller: no tuning
    *lat = *thr = std::min(s->p.fixed_team, max_team(s, n));
    return MEG_OK;
  }
  auto it = s->team.find(n);
  if (it != s->team.end()) {
    *lat = it->second.lat;
    *thr = it->second.thr;
    return MEG_OK;
  }
  const int pmax = max_team(s, n);
  std::vector<int> cand;
  for (int p = 1; p <= pmax; p *= 2) cand.push_back(p);
  if (cand.back() != pmax) cand.push_back(pmax);
  const bool single = cand.size() == 1;
  // synthetic instance: M = u u^T + 0.01 (G + G^T) / sqrt(2n), FP32
  SplitMix rng{0x7475756e65ull ^ (uint64_t)n};
  std::vector<double> u(n);
  double nu = 0.0;
  for (auto& v : u) {
    v = rng.normal();
    nu += v * v;
  }
  for (auto& v : u) v /= std::sqrt(nu);
  std::vector<float> M((size_t)n * n);
  const double sc = 0.01 / std::sqrt(2.0 * (double)n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i; j < n; ++j) {
      const double v = u[i] * u[j] + sc * (rng.normal() + rng.normal());
      M[(size_t)i * n + j] = M[(size_t)j * n + i] = (float)v;
    }
  float* dM = nullptr;
  if (hipMalloc((void**)&dM, M.size() * sizeof(float)) != hipSuccess) return fail(s);
  meg_status st = MEG_OK;
  if (hipMemcpy(dM, M.data(), M.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) st = fail(s);
  std::vector<double> tper(cand.size(), 1e30);
  for (size_t ci = 0; ci < cand.size() && st == MEG_OK; ++ci) {
    const int P = cand[ci];
    const Layout L = layout(n, P);
    size_t off = 0;
    if (!s->arena.alloc(L.bytes, &off)) continue;  // does not fit now: skip this size
    meg_request q{};
    q.kind = MEG_GRAD_DENOISE_DENSE;
    q.r = 4;
    q.n = n;
    q.M = dM;
    q.ld = n;
    q.q = 1;
    q.max_iters = 1 << 20;
    q.eta = 1.0;
    q.eps_scale = 0.8;
    q.eps_c = 10.0;
    q.eps_pow = 2.0;
    q.oversample = 4;
    q.max_inner = 3;
    const double lam = 1.0;
    st = setup_instance(s, q, u.data(), &lam, P, s->arena_base + off, L, 3, 3, &s->h_slots[kProbeSlot]);
    double ms = 0.0;
    if (st == MEG_OK) st = launch_serve(s, {kProbeSlot}, {2}, &ms);  // warm-up
    if (st == MEG_OK) st = launch_serve(s, {kProbeSlot}, {6}, &ms);
    if (st == MEG_OK) tper[ci] = ms / 6.0;
    s->h_slots[kProbeSlot] = Slot<float>{};
    s->arena.release(off, L.bytes);
  }
  (void)hipFree(dM);
  if (st != MEG_OK) return st;
  double best = 1e30;
  for (double t : tper) best = std::min(best, t);
  if (best >= 1e29) {  // no candidate fitted the arena now: a default, not cached
    *lat = *thr = single ? cand[0] : std::min(4, pmax);
    return MEG_OK;
  }
  int pl = cand.back(), pt = cand[0];
  for (size_t ci = 0; ci < cand.size(); ++ci)
    if (tper[ci] <= 1.15 * best) {
      pl = cand[ci];
      break;
    }
  double wbest = 1e30;
  for (size_t ci = 0; ci < cand.size(); ++ci)
    if (tper[ci] < 1e29 && cand[ci] * tper[ci] < wbest) {
      wbest = cand[ci] * tper[ci];
      pt = cand[ci];
    }
  Tuned tu;
  tu.lat = pl;
  tu.thr = pt;
  for (size_t ci = 0; ci < cand.size(); ++ci)
    if (tper[ci] < 1e29) tu.ms_per_step[cand[ci]] = tper[ci];
  s->team[n] = tu;
  *lat = pl;
  *thr = pt;
  return MEG_OK;
}

// retire every resident instance that stopped, failed or reached its cap
meg_status retire(meg_server s) {
  for (int sl = 0; sl < kMaxSlots; ++sl) {
    const int64_t id = s->slot_req[sl];
    if (id < 0) continue;
    Req& q = s->reqs[id];
    const SlotSummary& sm = s->h_sum[sl];
    q.iters = sm.t - 1;
    const bool bad = sm.status != 0 || sm.barerr != 0;
    if (!(bad || sm.stop || q.iters >= q.r.max_iters)) continue;
    const Slot<float>& slot = s->h_slots[sl];
    // results: control block and the basis block
    Ctl h;
    SCHK(s, hipMemcpy(&h, slot.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    const int64_t n = q.r.n;
    const int r = q.r.r;
    std::vector<float> B((size_t)n * kKB);
    const float* blk = h.src == 0 ? slot.Z0 : (h.src == 1 ? slot.Z1 : slot.Z2);
    SCHK(s, hipMemcpy(B.data(), blk, B.size() * sizeof(float), hipMemcpyDeviceToHost));
    q.V.assign((size_t)n * r, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int l = 0; l < r; ++l) {
        double v = 0.0;
        for (int c = 0; c < kKB; ++c) v += (double)B[(size_t)i * kKB + c] * h.Wb[c * kKB + l];
        q.V[(size_t)l * n + i] = v;
      }
    q.d.assign(h.d, h.d + r);
    q.alpha = h.alpha;
    q.applies = h.applies_done;
    const Info& in = h.info;
    meg_step_info& o = q.last;
    o.t = in.t;
    o.f = __builtin_nan("");
    o.eps_t = in.eps_t;
    o.cert_L = in.cert_L;
    o.cert_bound = in.cert_bound;
    o.cert_holds = in.cert_holds;
    o.inner_iters = in.inner_iters;
    o.ritz_gap = in.ritz_gap;
    o.resid_max = in.resid_max;
    o.mu_r1 = in.mu_r1;
    o.sigma = in.sigma;
    o.converged = in.converged;
    o.cert_resolved = in.cert_resolved;
    o.resid_r1 = in.resid_r1;
    o.cert_L_up = in.cert_L_up;
    o.mu_r1_up = in.mu_r1_up;
    q.iters = h.t - 1;
    q.state = bad ? 3 : 2;
    q.status = sm.barerr ? MEG_ERR_DEVICE : (sm.status ? sm.status : MEG_OK);
    q.t_done = now_ms(s);
    s->arena.release(q.off, q.bytes);
    s->free_wg += q.nwg;
    s->slot_req[sl] = -1;
    s->h_slots[sl] = Slot<float>{};
    std::memset(&s->h_sum[sl], 0, sizeof(SlotSummary));
    if (bad) ++s->failed_reqs; else ++s->completed;
  }
  return MEG_OK;
}

// admit queued requests in arrival order while a slot, a team and memory are free
meg_status admit(meg_server s) {
  int resident = 0;
  for (int sl = 0; sl < kMaxSlots; ++sl) resident += s->slot_req[sl] >= 0;
  bool any = false;
  while (!s->queue.empty() && resident < s->p.max_resident) {
    const int64_t id = s->queue.front();
    Req& q = s->reqs[id];
    int pl = 0, pt = 0;
    meg_status st = tune(s, q.r.n, &pl, &pt);
    if (st != MEG_OK) return st;
    const int P = s->queue.size() > 1 ? pt : pl;  // others waiting: the throughput choice
    if (P > s->free_wg) break;
    const Layout L = layout(q.r.n, P);
    size_t off = 0;
    if (!s->arena.alloc(L.bytes, &off)) break;
    int sl = 0;
    while (s->slot_req[sl] >= 0) ++sl;
    st = setup_instance(s, q.r, q.V0.data(), q.lam0.data(), P, s->arena_base + off, L, 1, q.r.max_inner,
                        &s->h_slots[sl]);
    if (st != MEG_OK) {
      s->arena.release(off, L.bytes);
      if (st == MEG_ERR_DEVICE) return st;
      q.state = 3;
      q.status = st;
      ++s->failed_reqs;
      s->queue.pop_front();
      continue;
    }
    q.slot = sl;
    q.nwg = P;
    q.step_ms = s->team.count(q.r.n) ? s->team[q.r.n].step_ms(P) : 1.0;
    q.off = off;
    q.bytes = L.bytes;
    q.state = 1;
    q.t_admit = now_ms(s);
    s->slot_req[sl] = id;
    s->free_wg -= P;
    s->queue.pop_front();
    ++resident;
    any = true;
  }
  // the planes are split from the caller's M: done before the request counts as admitted
  if (any) SCHK(s, hipStreamSynchronize(s->stream));
  return MEG_OK;
}

meg_status check_server(meg_server s) {
  if (!s) return MEG_ERR_INVALID_ARG;
  if (s->failed) return MEG_ERR_STATE;
  return MEG_OK;
}

}  // namespace

extern "C" {

meg_status meg_server_create(meg_server* out, const meg_server_params* params, void* stream) {
  if (!out || !params) return MEG_ERR_INVALID_ARG;
  *out = nullptr;
  if (params->launch_steps < 1 || params->launch_steps > 1024 || params->max_resident < 1 ||
      params->max_resident > kMaxSlots || params->budget_bytes < 0 || (params->flags & ~MEG_SERVER_FLAG_GRAPH) != 0 ||
      params->fixed_team < 0 || params->fixed_team > kBarGroupSize * kBarMaxGroups)
    return MEG_ERR_INVALID_ARG;
  int dev = 0, coop = 0, ncu = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, serve_kernel(), kNT, 0) != hipSuccess || occ < 1) {
    (void)hipGetLastError();
    return MEG_ERR_DEVICE;
  }
  if ((params->flags & MEG_SERVER_FLAG_GRAPH) && !stream) return MEG_ERR_INVALID_ARG;  // capture needs a stream
  meg_server s = new (std::nothrow) meg_server_s();
  if (!s) return MEG_ERR_OUT_OF_MEMORY;
  s->p = *params;
  s->stream = (hipStream_t)stream;
  s->capacity = std::min(ncu * occ, kBarGroupSize * kBarMaxGroups);
  s->free_wg = s->capacity;
  s->slot_req.assign(kMaxSlots, -1);
  const size_t budget = params->budget_bytes > 0 ? (size_t)params->budget_bytes : ((size_t)4 << 30);
  bool ok = hipMalloc((void**)&s->arena_base, budget) == hipSuccess &&
            hipMalloc((void**)&s->d_slots, sizeof(Slot<float>) * (kMaxSlots + 1)) == hipSuccess &&
            hipMalloc((void**)&s->d_team, sizeof(int2) * s->capacity) == hipSuccess &&
            hipMalloc((void**)&s->d_sum, sizeof(SlotSummary) * (kMaxSlots + 1)) == hipSuccess &&
            hipMalloc((void**)&s->d_prm, sizeof(ServeParams)) == hipSuccess &&
            hipHostMalloc((void**)&s->h_prm, sizeof(ServeParams)) == hipSuccess &&
            hipHostMalloc((void**)&s->h_slots, sizeof(Slot<float>) * (kMaxSlots + 1)) == hipSuccess &&
            hipHostMalloc((void**)&s->h_team, sizeof(int2) * s->capacity) == hipSuccess &&
            hipHostMalloc((void**)&s->h_sum, sizeof(SlotSummary) * (kMaxSlots + 1)) == hipSuccess &&
            hipEventCreate(&s->ev_a) == hipSuccess && hipEventCreate(&s->ev_b) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    meg_server_destroy(s);
    return MEG_ERR_OUT_OF_MEMORY;
  }
  s->arena.init(budget);
  for (int i = 0; i <= kMaxSlots; ++i) s->h_slots[i] = Slot<float>{};
  std::memset(s->h_sum, 0, sizeof(SlotSummary) * (kMaxSlots + 1));
  for (int k = 0; k < s->capacity; ++k) s->h_team[k] = make_int2(-1, 0);
  s->h_prm->seq = 0;
  s->h_prm->budget = 0;
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return MEG_OK;
}

meg_status meg_server_submit(meg_server s, const meg_request* req, int64_t* id) {
  meg_status st = check_server(s);
  if (st != MEG_OK) return st;
  if (!id) return MEG_ERR_INVALID_ARG;
  st = validate_request(req);
  if (st != MEG_OK) return st;
  // must fit the arena on its own (with the largest team it could get)
  if (layout(req->n, max_team(s, req->n)).bytes > s->arena.size) return MEG_ERR_OUT_OF_MEMORY;
  const int64_t k = s->next_id++;
  Req& q = s->reqs[k];
  q.r = *req;
  q.V0.assign(req->V0, req->V0 + (size_t)req->n * req->q);
  q.lam0.assign(req->lambda0, req->lambda0 + req->q);
  q.r.V0 = nullptr;
  q.r.lambda0 = nullptr;
  q.t_submit = now_ms(s);
  s->queue.push_back(k);
  ++s->submitted;
  *id = k;
  return MEG_OK;
}

meg_status meg_server_run(meg_server s, int32_t rounds, int32_t* pending) {
  meg_status st = check_server(s);
  if (st != MEG_OK) return st;
  if (rounds < 0) return MEG_ERR_INVALID_ARG;
  for (int rd = 0; rd < rounds; ++rd) {
    if ((st = retire(s)) != MEG_OK) return st;
    if ((st = admit(s)) != MEG_OK) return st;
    // Time budget of the launch: every team steps until it is used up (the
    // device clock decides at step boundaries), so the teams finish
    // together.  D = max(launch_steps x the fastest step, the slowest single
    // step) by the autotuner's times, raised to 0.9 of the last launch (the
    // autotuner times instances alone; under load steps take longer).
    std::vector<int> slots, steps;
    double tmin = 1e30, tmax = 0.0;
    for (int sl = 0; sl < kMaxSlots; ++sl) {
      const int64_t id = s->slot_req[sl];
      if (id < 0) continue;
      const Req& q = s->reqs[id];
      slots.push_back(sl);
      tmin = std::min(tmin, q.step_ms);
      tmax = std::max(tmax, q.step_ms);
    }
    if (slots.empty()) break;
    const double D = std::max({s->p.launch_steps * tmin, tmax, 0.9 * s->last_launch_ms});
    for (int sl : slots) {
      const Req& q = s->reqs[s->slot_req[sl]];
      steps.push_back((int)std::min<int64_t>((int64_t)s->p.launch_steps * 64, q.r.max_iters - q.iters));
    }
    double ms = 0.0;
    if ((st = launch_serve(s, slots, steps, &ms, D)) != MEG_OK) return st;
    ++s->launches;
    s->kernel_ms += ms;
    s->last_launch_ms = ms;
    for (size_t i = 0; i < slots.size(); ++i) {
      Req& q = s->reqs[s->slot_req[slots[i]]];
      const int64_t it = s->h_sum[slots[i]].t - 1;
      s->iterations += it - q.iters;
      q.iters = it;
    }
  }
  if ((st = retire(s)) != MEG_OK) return st;
  if (pending) {
    int res = 0;
    for (int sl = 0; sl < kMaxSlots; ++sl) res += s->slot_req[sl] >= 0;
    *pending = res + (int)s->queue.size();
  }
  return MEG_OK;
}

meg_status meg_server_query(meg_server s, int64_t id, meg_request_status* out) {
  if (!s || !out) return MEG_ERR_INVALID_ARG;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return MEG_ERR_INVALID_ARG;
  const Req& q = it->second;
  std::memset(out, 0, sizeof(*out));
  out->state = q.state;
  out->status = q.status;
  out->iterations = q.iters;
  out->submit_ms = q.t_submit;
  out->admit_ms = q.t_admit;
  out->done_ms = q.t_done;
  out->team = q.nwg;
  out->last = q.last;
  out->applies = q.applies;
  return MEG_OK;
}

meg_status meg_server_result(meg_server s, int64_t id, double* V, double* d, double* alpha) {
  if (!s) return MEG_ERR_INVALID_ARG;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return MEG_ERR_INVALID_ARG;
  const Req& q = it->second;
  if (q.state != 2) return MEG_ERR_STATE;
  if (V) std::memcpy(V, q.V.data(), q.V.size() * sizeof(double));
  if (d) std::memcpy(d, q.d.data(), q.d.size() * sizeof(double));
  if (alpha) *alpha = q.alpha;
  return MEG_OK;
}

meg_status meg_server_release(meg_server s, int64_t id) {
  if (!s) return MEG_ERR_INVALID_ARG;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return MEG_ERR_INVALID_ARG;
  if (it->second.state < 2) return MEG_ERR_STATE;
  s->reqs.erase(it);
  return MEG_OK;
}

meg_status meg_server_team(meg_server s, int64_t n, int32_t* latency_team, int32_t* throughput_team) {
  meg_status st = check_server(s);
  if (st != MEG_OK) return st;
  if (n < 16 || n > 32768) return MEG_ERR_INVALID_ARG;
  int pl = 0, pt = 0;
  st = tune(s, n, &pl, &pt);
  if (st != MEG_OK) return st;
  if (latency_team) *latency_team = pl;
  if (throughput_team) *throughput_team = pt;
  return MEG_OK;
}

meg_status meg_server_get_stats(meg_server s, meg_server_stats* out) {
  if (!s || !out) return MEG_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed_reqs;
  out->launches = s->launches;
  out->iterations = s->iterations;
  out->kernel_ms = s->kernel_ms;
  int res = 0;
  for (int sl = 0; sl < kMaxSlots; ++sl) res += s->slot_req[sl] >= 0;
  out->resident = res;
  out->queued = (int32_t)s->queue.size();
  out->capacity_wg = s->capacity;
  out->graph_node = s->graph_exec ? (s->graph_coop ? 1 : 2) : 0;
  out->arena_bytes = (int64_t)s->arena.size;
  out->arena_used = (int64_t)s->arena.used;
  out->arena_peak = (int64_t)s->arena.peak;
  return MEG_OK;
}

void meg_server_destroy(meg_server s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->d_prm) (void)hipFree(s->d_prm);
  if (s->h_prm) (void)hipHostFree(s->h_prm);
  if (s->arena_base) (void)hipFree(s->arena_base);
  if (s->d_slots) (void)hipFree(s->d_slots);
  if (s->d_team) (void)hipFree(s->d_team);
  if (s->d_sum) (void)hipFree(s->d_sum);
  if (s->h_slots) (void)hipHostFree(s->h_slots);
  if (s->h_team) (void)hipHostFree(s->h_team);
  if (s->h_sum) (void)hipHostFree(s->h_sum);
  if (s->ev_a) (void)hipEventDestroy(s->ev_a);
  if (s->ev_b) (void)hipEventDestroy(s->ev_b);
  delete s;
}

}  // extern "C"
