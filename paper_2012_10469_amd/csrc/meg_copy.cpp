// meg_copy: a plain device-to-device copy of a known size, the calibration
// reference for the HBM traffic counters (FETCH_SIZE, WRITE_SIZE) that are
// read for the step kernel: the counters' reading for this kernel divided by
// its exact byte count is the factor applied to the step kernel's readings.
//
//   meg_copy [MiB]   (default 1024): copies MiB mebibytes three times
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
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
  std::printf("{\"copy_bytes_read\": %zu, \"copy_bytes_written\": %zu, \"best_ms\": %.4f, \"gbs\": %.1f}\n", bytes,
              bytes, best, 2.0 * bytes / (best * 1e-3) / 1e9);
  (void)hipFree(a);
  (void)hipFree(b);
  return 0;
}
