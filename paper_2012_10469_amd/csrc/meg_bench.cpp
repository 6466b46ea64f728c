// meg_bench: native driver of the low-rank MEG library for profilers.
//
// Runs the masked matrix-completion workload (CSR mask, FP32 state), or the
// precision-form denoising workload (M as bf16 planes, FP32 state), through
// the C ABI only, without Python: warmup iterations, then a timed run of
// meg_solve launches, then one JSON line with the library's step-kernel
// counters (launches, iterations, operator applies, HIP-event GPU time) and
// the host wall clock.  `--trace P` then estimates tr exp(M_t) at the final
// iterate (meg_trace_exp, the solver block plus P seeded Gaussian probes,
// weight 1/P) `--trace-reps` times and adds the last call's estimate and
// the mean wall time per call.  The workload files are written by `bench.py
// --write-workload PATH` / `--write-dense-workload PATH` from the seeded
// generators the benchmark and the tests use.
//
// File layouts (little-endian):
//   "MEGW0001", int64 n, int64 nnz, int32 r, int32 q, int32 row_ptr[n+1],
//   int32 col[nnz], float val[nnz], double V0[n*q] (column-major), double lambda0[q];
//   "MEGD0001", int64 n, int64 ld, int32 r, int32 q, uint16 hi[n*ld],
//   uint16 lo[n*ld], double V0[n*q] (column-major), double lambda0[q];
//   "MEGB0001", int64 n, int64 m, int32 r, int32 q, double eta, float A[2m*n]
//   (rows a_1..a_m, b_1..b_m), float y[m], double V0[n*q], double lambda0[q]
//   (the recovery problem of the experiments: bilinear measurements, FP32 state).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "meg.h"

namespace {

struct Workload {
  bool dense = false;
  bool bilinear = false;
  double eta = 1.0;
  std::vector<float> A, y;
  int64_t n = 0, nnz = 0, ld = 0;
  int32_t r = 0, q = 0;
  std::vector<int32_t> row_ptr, col;
  std::vector<float> val;
  std::vector<uint16_t> hi, lo;
  std::vector<double> V0, lam0;
};

bool read_all(FILE* f, void* p, size_t bytes) { return bytes == 0 || std::fread(p, 1, bytes, f) == bytes; }

bool load(const char* path, Workload& w) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  char magic[8];
  bool ok = read_all(f, magic, 8);
  w.dense = ok && std::memcmp(magic, "MEGD0001", 8) == 0;
  w.bilinear = ok && std::memcmp(magic, "MEGB0001", 8) == 0;
  if (w.bilinear) {  // n, m (kept in nnz), r, q, eta, A, y
    ok = read_all(f, &w.n, 8) && read_all(f, &w.nnz, 8) && read_all(f, &w.r, 4) && read_all(f, &w.q, 4) &&
         read_all(f, &w.eta, 8);
    ok = ok && w.n > 0 && w.n < (int64_t)1 << 20 && w.nnz >= 1 && w.nnz < (int64_t)1 << 28 && w.r >= 1 &&
         w.q >= 1 && w.q <= w.r && w.eta > 0.0;
    if (ok) {
      w.A.resize((size_t)2 * w.nnz * w.n);
      w.y.resize(w.nnz);
      ok = read_all(f, w.A.data(), w.A.size() * 4) && read_all(f, w.y.data(), w.y.size() * 4);
    }
    if (ok) {
      w.V0.resize((size_t)w.n * w.q);
      w.lam0.resize(w.q);
      ok = read_all(f, w.V0.data(), w.V0.size() * 8) && read_all(f, w.lam0.data(), w.lam0.size() * 8);
    }
    std::fclose(f);
    return ok;
  }
  ok = ok && (w.dense || std::memcmp(magic, "MEGW0001", 8) == 0) && read_all(f, &w.n, 8) &&
       read_all(f, w.dense ? &w.ld : &w.nnz, 8) && read_all(f, &w.r, 4) && read_all(f, &w.q, 4);
  ok = ok && w.n > 0 && w.nnz >= 0 && w.r >= 1 && w.q >= 1 && w.q <= w.r && w.n < (int64_t)1 << 31 &&
       w.nnz < (int64_t)1 << 31 && (!w.dense || (w.ld >= w.n && w.ld < (int64_t)1 << 31));
  if (ok && w.dense) {
    w.hi.resize((size_t)w.n * w.ld);
    w.lo.resize((size_t)w.n * w.ld);
    ok = read_all(f, w.hi.data(), w.hi.size() * 2) && read_all(f, w.lo.data(), w.lo.size() * 2);
  } else if (ok) {
    w.row_ptr.resize(w.n + 1);
    w.col.resize(w.nnz);
    w.val.resize(w.nnz);
    ok = read_all(f, w.row_ptr.data(), w.row_ptr.size() * 4) && read_all(f, w.col.data(), w.col.size() * 4) &&
         read_all(f, w.val.data(), w.val.size() * 4);
  }
  if (ok) {
    w.V0.resize((size_t)w.n * w.q);
    w.lam0.resize(w.q);
    ok = read_all(f, w.V0.data(), w.V0.size() * 8) && read_all(f, w.lam0.data(), w.lam0.size() * 8);
  }
  std::fclose(f);
  return ok;
}

template <typename T>
T* to_device(const std::vector<T>& h) {
  T* d = nullptr;
  if (hipMalloc((void**)&d, std::max<size_t>(h.size(), 1) * sizeof(T)) != hipSuccess) return nullptr;
  if (!h.empty() && hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  return d;
}

int fail(const char* what, int code) {
  std::fprintf(stderr, "meg_bench: %s\n", what);
  return code;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2)
    return fail("usage: meg_bench WORKLOAD [--steps K] [--warmup W] [--launch-steps L] [--max-inner M] [--trace P] "
                "[--trace-reps R]", 2);
  int64_t steps = 512, warmup = 64, launch = 64;
  int max_inner = 12, trace_p = -1, trace_reps = 3;
  for (int i = 2; i + 1 < argc; i += 2) {
    const std::string a = argv[i];
    const long long v = std::atoll(argv[i + 1]);
    if (a == "--steps") steps = v;
    else if (a == "--warmup") warmup = v;
    else if (a == "--launch-steps") launch = v;
    else if (a == "--max-inner") max_inner = (int)v;
    else if (a == "--trace") trace_p = (int)v;
    else if (a == "--trace-reps") trace_reps = (int)v;
    else return fail("unknown option", 2);
  }
  if (steps < 1 || warmup < 0 || launch < 1 || max_inner < 1 || max_inner > 64 || trace_p > 4096 || trace_reps < 1)
    return fail("bad option value", 2);

  Workload w;
  if (!load(argv[1], w)) return fail("cannot read workload file", 2);
  std::fprintf(stderr, "[meg_bench] %s n=%lld nnz=%lld ld=%lld r=%d q=%d\n", w.bilinear ? "bilinear measurements (nnz = m)" : (w.dense ? "dense bf16 planes" : "csr"),
               (long long)w.n, (long long)w.nnz, (long long)w.ld, w.r, w.q);

  int32_t* d_rp = nullptr;
  int32_t* d_col = nullptr;
  float* d_val = nullptr;
  uint16_t* d_hi = nullptr;
  uint16_t* d_lo = nullptr;
  float* d_A = nullptr;
  float* d_y = nullptr;
  if (w.bilinear) {
    d_A = to_device(w.A);
    d_y = to_device(w.y);
    if (!d_A || !d_y) return fail("device allocation or copy failed", 3);
    std::vector<float>().swap(w.A);
  } else if (w.dense) {
    d_hi = to_device(w.hi);
    d_lo = to_device(w.lo);
    if (!d_hi || !d_lo) return fail("device allocation or copy failed", 3);
    std::vector<uint16_t>().swap(w.hi);
    std::vector<uint16_t>().swap(w.lo);
  } else {
    d_rp = to_device(w.row_ptr);
    d_col = to_device(w.col);
    d_val = to_device(w.val);
    if (!d_rp || !d_col || !d_val) return fail("device allocation or copy failed", 3);
  }
  hipStream_t stream = nullptr;
  if (hipStreamCreate(&stream) != hipSuccess) return fail("hipStreamCreate failed", 3);

  meg_params p;
  std::memset(&p, 0, sizeof(p));
  p.n = w.n;
  p.r = w.r;
  p.oversample = 4;
  p.prec = w.dense ? MEG_PREC_F32_BF16X3 : MEG_PREC_F32;
  p.min_inner = 1;
  p.max_inner = max_inner;
  p.eta = w.bilinear ? w.eta : 1.0;
  p.eps_scale = 0.8;
  p.eps_c = 10.0;
  p.eps_pow = 2.0;
  p.seed = 0;
  meg_objective o;
  std::memset(&o, 0, sizeof(o));
  if (w.bilinear) {
    o.kind = MEG_GRAD_BILINEAR;
    o.A = d_A;
    o.lda = w.n;
    o.b = d_y;
    o.m = w.nnz;
  } else if (w.dense) {
    o.kind = MEG_GRAD_DENOISE_DENSE;
    o.dense = d_hi;
    o.dense_lo = d_lo;
    o.ld = w.ld;
  } else {
    o.kind = MEG_GRAD_MASKED_CSR;
    o.row_ptr = d_rp;
    o.col = d_col;
    o.val = d_val;
    o.nnz = w.nnz;
  }
  meg_start s;
  std::memset(&s, 0, sizeof(s));
  s.q = w.q;
  s.V0 = w.V0.data();
  s.lambda0 = w.lam0.data();

  meg_ctx ctx = nullptr;
  meg_status st = meg_init(&ctx, &p, &o, &s, (void*)stream);
  if (st != MEG_OK) return fail(meg_status_str(st), 4);
  auto run = [&](int64_t iters) -> meg_status {
    for (int64_t done = 0; done < iters;) {
      const int64_t m = std::min(launch, iters - done);
      const meg_status e = meg_solve(ctx, m, 0.0, nullptr);
      if (e != MEG_OK) return e;
      done += m;
    }
    return MEG_OK;
  };
  std::fprintf(stderr, "[meg_bench] warmup %lld\n", (long long)warmup);
  if ((st = run(warmup)) != MEG_OK) return fail(meg_status_str(st), 5);
  meg_counters c;
  if ((st = meg_get_counters(ctx, &c, 1)) != MEG_OK) return fail(meg_status_str(st), 5);
  std::fprintf(stderr, "[meg_bench] timing %lld steps, %lld per launch\n", (long long)steps, (long long)launch);
  const auto t0 = std::chrono::steady_clock::now();
  if ((st = run(steps)) != MEG_OK) return fail(meg_status_str(st), 5);
  if (hipStreamSynchronize(stream) != hipSuccess) return fail("hipStreamSynchronize failed", 5);
  const auto t1 = std::chrono::steady_clock::now();
  if ((st = meg_get_counters(ctx, &c, 0)) != MEG_OK) return fail(meg_status_str(st), 5);
  meg_step_info info;
  if ((st = meg_certificate(ctx, &info)) != MEG_OK) return fail(meg_status_str(st), 5);
  const double wall_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  meg_trace_info tr;
  std::memset(&tr, 0, sizeof(tr));
  double trace_ms = 0.0;
  if (trace_p >= 0) {
    std::vector<double> U((size_t)w.n * std::max(trace_p, 1));
    std::mt19937_64 gen(17);
    std::normal_distribution<double> nd;
    for (double& u : U) u = nd(gen);
    double* d_u = nullptr;
    if (hipMalloc((void**)&d_u, U.size() * 8) != hipSuccess ||
        hipMemcpy(d_u, U.data(), U.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return fail("probe upload failed", 6);
    std::fprintf(stderr, "[meg_bench] trace estimate: %d probes, %d calls\n", trace_p, trace_reps);
    for (int rep = 0; rep < trace_reps; ++rep) {
      const auto a0 = std::chrono::steady_clock::now();
      st = meg_trace_exp(ctx, d_u, trace_p, trace_p > 0 ? 1.0 / trace_p : 1.0, 64, 1e-8, &tr);
      const auto a1 = std::chrono::steady_clock::now();
      if (st != MEG_OK) return fail(meg_status_str(st), 6);
      if (rep > 0 || trace_reps == 1) trace_ms += std::chrono::duration<double, std::milli>(a1 - a0).count();
    }
    trace_ms /= (trace_reps > 1 ? trace_reps - 1 : 1);
    (void)hipFree(d_u);
  }
  std::printf(
      "{\"workload\": \"%s\", \"n\": %lld, \"nnz\": %lld, \"r\": %d, \"steps\": %lld, "
      "\"launch_steps\": %lld, \"launches\": %lld, \"iterations\": %lld, \"applies\": %lld, \"workgroups\": %d, "
      "\"kernel_ms\": %.6f, \"avg_launch_us\": %.3f, \"wall_ms_per_step\": %.6f, \"iter_per_s\": %.3f, "
      "\"t\": %lld, \"cert_L\": %.6e, \"eps_t\": %.6e, \"trace_probes\": %d, \"trace_log_b\": %.10e, "
      "\"trace_steps\": %d, \"trace_ms_per_call\": %.4f}\n",
      w.bilinear ? "recovery_bilinear" : (w.dense ? "denoise_bf16x3" : "matrix_completion_csr"), (long long)w.n, (long long)w.nnz, w.r, (long long)steps, (long long)launch, (long long)c.launches,
      (long long)c.iterations, (long long)c.applies, c.workgroups, c.kernel_ms,
      c.launches ? 1e3 * c.kernel_ms / (double)c.launches : 0.0, wall_ms / (double)steps,
      1e3 * (double)steps / wall_ms, (long long)info.t, info.cert_L, info.eps_t, trace_p, tr.log_b, tr.steps,
      trace_ms);
  std::fflush(stdout);
  meg_destroy(ctx);
  (void)hipStreamDestroy(stream);
  for (void* q : {(void*)d_rp, (void*)d_col, (void*)d_val, (void*)d_hi, (void*)d_lo, (void*)d_A, (void*)d_y})
    if (q) (void)hipFree(q);
  return 0;
}
