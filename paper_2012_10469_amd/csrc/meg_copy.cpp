// meg_copy: a plain device-to-device copy of a known size, the calibration
// reference for the HBM traffic counters (FETCH_SIZE, WRITE_SIZE) that are
// read for the step kernel: the counters' reading for this kernel divided by
// its exact byte count is the factor applied to the step kernel's readings.
// It also prints the copy rate (bytes read + written per second) and a
// read-only streaming rate, the measured ceilings quoted beside HBM's peak.
//
//   meg_copy [MiB]   (default 1024): copies MiB mebibytes three times
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

// Read-only streaming rate: one contiguous slice per workgroup (512 threads,
// one workgroup per CU at 256 workgroups), four 16-byte loads per thread in
// flight; a per-thread sum keeps the loads.
__global__ __launch_bounds__(512) void k_read(const float4* __restrict__ src, size_t per_wg, float* __restrict__ out) {
  const float4* p = src + (size_t)blockIdx.x * per_wg;
  float acc = 0.f;
  for (size_t i0 = 0; i0 < per_wg; i0 += 4 * 512) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t i = i0 + (size_t)u * 512 + threadIdx.x;
      v[u] = i < per_wg ? p[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
  }
  out[(size_t)blockIdx.x * 512 + threadIdx.x] = acc;
}

int main(int argc, char** argv) {
  const size_t mib = argc > 1 ? (size_t)std::atoll(argv[1]) : 1024;
  if (mib < 1 || mib > 65536) {
    std::fprintf(stderr, "meg_copy: size out of range\n");
    return 2;
  }
  const size_t bytes = mib << 20, n = bytes / sizeof(float4);
  float4 *a = nullptr, *b = nullptr;
  if (hipMalloc((void**)&a, bytes) != hipSuccess || hipMalloc((void**)&b, bytes) != hipSuccess) {
    std::fprintf(stderr, "meg_copy: allocation failed\n");
    return 3;
  }
  if (hipMemset(a, 0, bytes) != hipSuccess) return 3;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 3;
  float best = 1e30f;
  for (int rep = 0; rep < 3; ++rep) {
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_copy, dim3(8192), dim3(256), 0, nullptr, a, b, n);
    hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) return 4;
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) best = ms;
  }
  // read-only rate over the same buffer, 256 workgroups
  float* sink = nullptr;
  if (hipMalloc((void**)&sink, (size_t)256 * 512 * sizeof(float)) != hipSuccess) return 3;
  const size_t per_wg = n / 256;
  float best_r = 1e30f;
  for (int rep = 0; rep < 3; ++rep) {
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_read, dim3(256), dim3(512), 0, nullptr, a, per_wg, sink);
    hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) return 4;
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_r) best_r = ms;
  }
  const double rbytes = (double)per_wg * 256 * sizeof(float4);
  std::printf("{\"copy_bytes_read\": %zu, \"copy_bytes_written\": %zu, \"best_ms\": %.4f, \"gbs\": %.1f, "
              "\"read_only_gbs\": %.1f}\n",
              bytes, bytes, best, 2.0 * bytes / (best * 1e-3) / 1e9, rbytes / (best_r * 1e-3) / 1e9);
  (void)hipFree(sink);
  (void)hipFree(a);
  (void)hipFree(b);
  return 0;
}
