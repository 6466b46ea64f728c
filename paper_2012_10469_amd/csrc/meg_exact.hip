// Exact MEG (Algorithm 1) on the GPU, as the comparison baseline of the
// low-rank method (the exact-versus-low-rank comparison of Section 7).
//
// With a constant step size the iterates of Algorithm 1 satisfy
//   log W_{t+1} = log W_t - eta grad f(W_t) - log tr(...) I,
// so W_{t+1} = exp(Y_{t+1}) / tr exp(Y_{t+1}) with Y_1 = log W_1 and
// Y_{t+1} = Y_t - eta grad f(W_t): the identity terms cancel in the
// normalisation and no matrix logarithm is needed after the start.  Each
// step forms grad f(W_t) and updates Y (one pass), then exp(Y - m I) by
// scaling and squaring: m and the scaling from Gershgorin bounds of Y, a
// degree-12 Taylor polynomial of (Y - m I) / 2^s by Horner's rule, s
// squarings.  Dense n x n FP64 throughout; the products are plain GEMMs
// (rocBLAS).  W_1 = (1 - eps_0) X_0 + (eps_0 / n) I is the low-rank method's
// first iterate, so both runs start from the same matrix.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/meg.h"

namespace {

constexpr int kTaylor = 12;

struct Sums {  // per-workgroup partials of the update pass
  double f, up, lo;
};

// f(W) and grad f(W) = C or W - M; Y <- Y - eta G; per-row Gershgorin
// bounds of the new Y (upper: Y_ii + sum_{j != i} |Y_ij|, lower: Y_ii - ...).
// One workgroup per row.
__global__ __launch_bounds__(256) void k_ex_update(int64_t n, int kind, const double* __restrict__ D, int64_t ld,
                                                   const double* __restrict__ W, double eta, double* __restrict__ Y,
                                                   Sums* __restrict__ part) {
  __shared__ double sr[3][4];
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double f = 0.0, off = 0.0, dia = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const double w = W[i * n + j], d = D[i * ld + j];
    double g;
    if (kind == MEG_GRAD_LINEAR_DENSE) {
      g = d;
      f += d * w;
    } else {
      g = w - d;
      f += 0.5 * g * g;
    }
    const double y = Y[i * n + j] - eta * g;
    Y[i * n + j] = y;
    if (i == j) dia = y; else off += fabs(y);
  }
  double v[3] = {f, off, dia};
  for (int q = 0; q < 3; ++q) {
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if (lane == 0) sr[q][wave] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double fs = (sr[0][0] + sr[0][1]) + (sr[0][2] + sr[0][3]);
    const double os = (sr[1][0] + sr[1][1]) + (sr[1][2] + sr[1][3]);
    const double ds = (sr[2][0] + sr[2][1]) + (sr[2][2] + sr[2][3]);
    part[i] = Sums{fs, ds + os, ds - os};
  }
}

// A = (Y - m I) / 2^s and E = I + A / kTaylor (the innermost Horner level)
__global__ __launch_bounds__(256) void k_ex_scale(int64_t n, const double* __restrict__ Y, double m, double sc,
                                                  double* __restrict__ A, double* __restrict__ E) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * 256) {
    const bool diag = (e / n) == (e % n);
    const double a = (Y[e] - (diag ? m : 0.0)) * sc;
    A[e] = a;
    E[e] = (diag ? 1.0 : 0.0) + a / kTaylor;
  }
}

// E = I + P / k (one Horner level: P = A E_previous)
__global__ __launch_bounds__(256) void k_ex_horner(int64_t n, const double* __restrict__ P, double ik,
                                                   double* __restrict__ E) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * 256)
    E[e] = ((e / n) == (e % n) ? 1.0 : 0.0) + P[e] * ik;
}

// out[b] = partial sums of the diagonal (b-th slice), for tr E
__global__ __launch_bounds__(256) void k_ex_trace(int64_t n, const double* __restrict__ E, double* __restrict__ out) {
  __shared__ double sr[4];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a += E[i * n + i];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) sr[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (sr[0] + sr[1]) + (sr[2] + sr[3]);
}

// W = (E + E^T) / (2 tr E)
__global__ __launch_bounds__(256) void k_ex_norm(int64_t n, const double* __restrict__ E, double itr,
                                                 double* __restrict__ W) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e % n;
    W[e] = 0.5 * (E[i * n + j] + E[j * n + i]) * itr;
  }
}

// out[b] = partial sums of a . b over slices (dot of two n*n matrices, or of
// two n x r blocks when cnt = n r)
__global__ __launch_bounds__(256) void k_ex_dot(int64_t cnt, const double* __restrict__ a,
                                                const double* __restrict__ b, double* __restrict__ out) {
  __shared__ double sr[4];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) s += a[e] * b[e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sr[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (sr[0] + sr[1]) + (sr[2] + sr[3]);
}

}  // namespace

struct meg_exact_s {
  int64_t n = 0;
  int kind = 0;
  const double* D = nullptr;  // C or M (borrowed)
  int64_t ld = 0;
  double eta = 1.0;
  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  double *Y = nullptr, *W = nullptr, *E = nullptr, *A = nullptr, *P = nullptr;
  void* part = nullptr;       // n Sums, or the slices of a reduction
  double* red = nullptr;      // host-visible partial copy
  int64_t t = 1;
  double m = 0.0, log_tr = 0.0;  // W = exp(Y - m I) / tr, log tr of that exponential
  bool failed = false;
};

namespace {

constexpr int kRedWg = 256;

meg_status ex_fail(meg_exact h) {
  h->failed = true;
  return MEG_ERR_DEVICE;
}

#define EXCHK(h, x)                                  \
  do {                                               \
    if ((x) != hipSuccess) return ex_fail(h);        \
  } while (0)
#define BLASCHK(h, x)                                         \
  do {                                                        \
    if ((x) != rocblas_status_success) return ex_fail(h);     \
  } while (0)

int grid_for(int64_t cnt) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (cnt + 255) / 256)); }

// C = A B for n x n row-major matrices (column-major GEMM of the transposes)
rocblas_status gemm(meg_exact h, const double* A, const double* B, double* C, int64_t rowsA) {
  const double one = 1.0, zero = 0.0;
  const rocblas_int n = (rocblas_int)h->n, m = (rocblas_int)rowsA;
  // row-major C (m x n) = A (m x n) B (n x n)  <=>  column-major C^T = B^T A^T
  return rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, n, m, n, &one, B, n, A, n, &zero, C,
                       n);
}

// sum of the kRedWg partials written by the last reduction kernel
meg_status reduce_sum(meg_exact h, double* out) {
  EXCHK(h, hipMemcpyAsync(h->red, h->part, kRedWg * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  EXCHK(h, hipStreamSynchronize(h->stream));
  double s = 0.0;
  for (int b = 0; b < kRedWg; ++b) s += h->red[b];
  *out = s;
  return MEG_OK;
}

// W = exp(Y - m I) / tr with m, s from the Gershgorin bounds [lo, up] of Y
meg_status exp_normalise(meg_exact h, double lo, double up) {
  const int64_t n = h->n, nn = n * n;
  const double spread = std::max(up - lo, 0.0);
  int s = 0;
  while (spread / std::ldexp(1.0, s) > 0.25 && s < 60) ++s;
  h->m = up;
  hipLaunchKernelGGL(k_ex_scale, dim3(grid_for(nn)), dim3(256), 0, h->stream, n, (const double*)h->Y, up,
                     std::ldexp(1.0, -s), h->A, h->E);
  EXCHK(h, hipGetLastError());
  for (int k = kTaylor - 1; k >= 1; --k) {  // E <- I + A E / k
    BLASCHK(h, gemm(h, h->A, h->E, h->P, n));
    hipLaunchKernelGGL(k_ex_horner, dim3(grid_for(nn)), dim3(256), 0, h->stream, n, (const double*)h->P,
                       1.0 / k, h->E);
    EXCHK(h, hipGetLastError());
  }
  for (int q = 0; q < s; ++q) {  // E <- E^2
    BLASCHK(h, gemm(h, h->E, h->E, h->P, n));
    std::swap(h->E, h->P);
  }
  hipLaunchKernelGGL(k_ex_trace, dim3(kRedWg), dim3(256), 0, h->stream, n, (const double*)h->E, (double*)h->part);
  EXCHK(h, hipGetLastError());
  double tr = 0.0;
  meg_status st = reduce_sum(h, &tr);
  if (st != MEG_OK) return st;
  if (!(tr > 0.0) || !std::isfinite(tr)) return MEG_ERR_NUMERIC;
  h->log_tr = std::log(tr);
  hipLaunchKernelGGL(k_ex_norm, dim3(grid_for(nn)), dim3(256), 0, h->stream, n, (const double*)h->E, 1.0 / tr, h->W);
  EXCHK(h, hipGetLastError());
  return MEG_OK;
}

void ex_free(meg_exact h) {
  if (!h) return;
  for (void* p : {(void*)h->Y, (void*)h->W, (void*)h->E, (void*)h->A, (void*)h->P, h->part})
    if (p) (void)hipFree(p);
  if (h->red) (void)hipHostFree(h->red);
  if (h->blas) (void)rocblas_destroy_handle(h->blas);
  delete h;
}

}  // namespace

extern "C" {

meg_status meg_exact_create(meg_exact* out, const meg_params* p, const meg_objective* obj, const meg_start* start,
                            void* stream) {
  if (!out) return MEG_ERR_INVALID_ARG;
  *out = nullptr;
  if (!p || !obj || !start || !start->V0 || !start->lambda0) return MEG_ERR_INVALID_ARG;
  const int64_t n = p->n;
  if (n < 2 || n > 8192 || p->prec != MEG_PREC_F64 || !(p->eta > 0.0)) return MEG_ERR_INVALID_ARG;
  if (obj->kind != MEG_GRAD_LINEAR_DENSE && obj->kind != MEG_GRAD_DENOISE_DENSE) return MEG_ERR_UNSUPPORTED;
  if (!obj->dense || obj->ld < n || start->q < 1 || start->q > n) return MEG_ERR_INVALID_ARG;
  const double eps0 = p->eps_scale / std::pow(p->eps_c + 1.0, p->eps_pow);
  if (!(eps0 > 0.0 && eps0 <= 0.75)) return MEG_ERR_INVALID_ARG;
  double lsum = 0.0;
  for (int l = 0; l < start->q; ++l) {
    if (!(start->lambda0[l] >= 0.0)) return MEG_ERR_INVALID_ARG;
    lsum += start->lambda0[l];
  }
  if (std::fabs(lsum - 1.0) > 1e-8) return MEG_ERR_INVALID_ARG;
  meg_exact h = new (std::nothrow) meg_exact_s();
  if (!h) return MEG_ERR_OUT_OF_MEMORY;
  h->n = n;
  h->kind = obj->kind;
  h->D = (const double*)obj->dense;
  h->ld = obj->ld;
  h->eta = p->eta;
  h->stream = (hipStream_t)stream;
  const size_t nn = (size_t)n * n;
  bool ok = hipMalloc((void**)&h->Y, nn * 8) == hipSuccess && hipMalloc((void**)&h->W, nn * 8) == hipSuccess &&
            hipMalloc((void**)&h->E, nn * 8) == hipSuccess && hipMalloc((void**)&h->A, nn * 8) == hipSuccess &&
            hipMalloc((void**)&h->P, nn * 8) == hipSuccess &&
            hipMalloc(&h->part, std::max<size_t>((size_t)n, kRedWg) * sizeof(Sums)) == hipSuccess &&
            hipHostMalloc((void**)&h->red, std::max<size_t>((size_t)n, kRedWg) * sizeof(Sums)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    ex_free(h);
    return MEG_ERR_OUT_OF_MEMORY;
  }
  if (rocblas_create_handle(&h->blas) != rocblas_status_success ||
      rocblas_set_stream(h->blas, h->stream) != rocblas_status_success) {
    ex_free(h);
    return MEG_ERR_DEVICE;
  }
  // W_1 = (1 - eps_0) X_0 + (eps_0/n) I and Y_1 = log W_1 in closed form: with
  // an orthonormal V0, log W_1 = log(a) I + V0 diag(log(a + (1-eps_0) lambda0) - log a) V0^T, a = eps_0/n
  const int q = start->q;
  std::vector<double> Q((size_t)n * q);
  for (int l = 0; l < q; ++l)
    for (int64_t i = 0; i < n; ++i) Q[(size_t)i * q + l] = start->V0[(size_t)l * n + i];
  for (int a = 0; a < q; ++a)  // orthonormal columns
    for (int b = a; b < q; ++b) {
      double dot = 0.0;
      for (int64_t i = 0; i < n; ++i) dot += Q[(size_t)i * q + a] * Q[(size_t)i * q + b];
      if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-8) {
        ex_free(h);
        return MEG_ERR_INVALID_ARG;
      }
    }
  const double a0 = eps0 / (double)n, la = std::log(a0);
  std::vector<double> wv(q), lv(q), Wh(nn), Yh(nn);
  for (int l = 0; l < q; ++l) {
    wv[l] = (1.0 - eps0) * start->lambda0[l];
    lv[l] = std::log(a0 + wv[l]) - la;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double w = (i == j) ? a0 : 0.0, y = (i == j) ? la : 0.0;
      for (int l = 0; l < q; ++l) {
        const double vv = Q[(size_t)i * q + l] * Q[(size_t)j * q + l];
        w += wv[l] * vv;
        y += lv[l] * vv;
      }
      Wh[(size_t)i * n + j] = w;
      Yh[(size_t)i * n + j] = y;
    }
  if (hipMemcpyAsync(h->W, Wh.data(), nn * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemcpyAsync(h->Y, Yh.data(), nn * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    ex_free(h);
    return MEG_ERR_DEVICE;
  }
  // m and tr for the Bregman distance at t = 1 (W_1 = exp(Y_1) exactly)
  h->m = 0.0;
  h->log_tr = 0.0;
  *out = h;
  return MEG_OK;
}

meg_status meg_exact_step(meg_exact h, meg_exact_info* info) {
  if (!h) return MEG_ERR_INVALID_ARG;
  if (h->failed) return MEG_ERR_STATE;
  const int64_t n = h->n;
  hipLaunchKernelGGL(k_ex_update, dim3(n), dim3(256), 0, h->stream, n, h->kind, h->D, h->ld, (const double*)h->W,
                     h->eta, h->Y, (Sums*)h->part);
  EXCHK(h, hipGetLastError());
  EXCHK(h, hipMemcpyAsync(h->red, h->part, n * sizeof(Sums), hipMemcpyDeviceToHost, h->stream));
  EXCHK(h, hipStreamSynchronize(h->stream));
  const Sums* ps = (const Sums*)h->red;
  double f = 0.0, up = -INFINITY, lo = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    f += ps[i].f;
    up = std::max(up, ps[i].up);
    lo = std::min(lo, ps[i].lo);
  }
  meg_status st = exp_normalise(h, lo, up);
  if (st != MEG_OK) return st;
  EXCHK(h, hipStreamSynchronize(h->stream));
  if (info) {
    info->t = h->t;
    info->f = f;
  }
  ++h->t;
  return MEG_OK;
}

meg_status meg_exact_get(meg_exact h, double* W, int64_t* t) {
  if (!h) return MEG_ERR_INVALID_ARG;
  if (h->failed) return MEG_ERR_STATE;
  if (W) {
    EXCHK(h, hipMemcpyAsync(W, h->W, (size_t)h->n * h->n * 8, hipMemcpyDeviceToHost, h->stream));
    EXCHK(h, hipStreamSynchronize(h->stream));
  }
  if (t) *t = h->t;
  return MEG_OK;
}

meg_status meg_exact_bregman(meg_exact h, const double* V, int32_t r, const double* d, double alpha, double* out) {
  if (!h || !V || !d || !out || r < 1 || r >= h->n || !(alpha > 0.0)) return MEG_ERR_INVALID_ARG;
  if (h->failed) return MEG_ERR_STATE;
  for (int l = 0; l < r; ++l)
    if (!(alpha + d[l] > 0.0)) return MEG_ERR_INVALID_ARG;
  const int64_t n = h->n;
  meg_status st = MEG_OK;
  // B(W, X) = tr(W log W) - tr(W log X), tr W = 1:
  //   tr(W log W) = tr(W Y) - m - log tr exp(Y - m I),
  //   tr(W log X) = log alpha + sum_l c_l v_l^T W v_l,  c_l = log(alpha + d_l) - log alpha
  hipLaunchKernelGGL(k_ex_dot, dim3(kRedWg), dim3(256), 0, h->stream, n * n, (const double*)h->W,
                     (const double*)h->Y, (double*)h->part);
  EXCHK(h, hipGetLastError());
  double wy = 0.0;
  st = reduce_sum(h, &wy);
  if (st != MEG_OK) return st;
  std::vector<double> Vr((size_t)n * r);  // row-major n x r
  for (int l = 0; l < r; ++l)
    for (int64_t i = 0; i < n; ++i) Vr[(size_t)i * r + l] = V[(size_t)l * n + i];
  EXCHK(h, hipMemcpyAsync(h->A, Vr.data(), Vr.size() * 8, hipMemcpyHostToDevice, h->stream));
  {  // P = W V (row-major n x r): column-major P^T (r x n) = V^T (r x n) W^T
    const double one = 1.0, zero = 0.0;
    BLASCHK(h, rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)r, (rocblas_int)n,
                             (rocblas_int)n, &one, h->A, (rocblas_int)r, h->W, (rocblas_int)n, &zero, h->P,
                             (rocblas_int)r));
  }
  std::vector<double> WV((size_t)n * r);
  EXCHK(h, hipMemcpyAsync(WV.data(), h->P, WV.size() * 8, hipMemcpyDeviceToHost, h->stream));
  EXCHK(h, hipStreamSynchronize(h->stream));
  double wlx = std::log(alpha);
  for (int l = 0; l < r; ++l) {
    double q = 0.0;
    for (int64_t i = 0; i < n; ++i) q += Vr[(size_t)i * r + l] * WV[(size_t)i * r + l];
    wlx += (std::log(alpha + d[l]) - std::log(alpha)) * q;
  }
  *out = (wy - h->m - h->log_tr) - wlx;
  return MEG_OK;
}

void meg_exact_destroy(meg_exact h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  ex_free(h);
}

}  // extern "C"
