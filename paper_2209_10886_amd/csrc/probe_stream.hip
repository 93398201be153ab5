// HBM calibration probe (diagnostic program, not part of libhbj).
//
//  1. streaming reads: G workgroups each read their own contiguous chunk (8 independent 32-byte
//     loads in flight per thread); prints aggregate and per-workgroup GB/s for G = 1 .. 2048;
//  2. a plain copy of 1 GiB (the reference kernel whose FETCH_SIZE / WRITE_SIZE counters calibrate
//     the counter-based traffic figures of the solver kernels).
#include <hip/hip_runtime.h>

#include <cstdio>

__global__ __launch_bounds__(512) void k_stream_read(const double4* __restrict__ a, size_t per4, double* out) {
  const double4* p = a + (size_t)blockIdx.x * per4;
  double s = 0;
  for (size_t i = threadIdx.x; i < per4; i += (size_t)blockDim.x * 8) {
    double4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t j = i + (size_t)k * blockDim.x;
      v[k] = (j < per4) ? p[j] : make_double4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k].x + v[k].y + v[k].z + v[k].w;
  }
  if (s == 12345.678) out[0] = s;  // keeps the loads alive
}

__global__ void k_plain_copy(const double4* __restrict__ a, double4* __restrict__ b, size_t n4) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) b[i] = a[i];
}

#define CHECK(x)                                                              \
  do {                                                                        \
    if ((x) != hipSuccess) {                                                  \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString((x)));    \
      return 1;                                                               \
    }                                                                         \
  } while (0)

int main() {
  const size_t total = (size_t)2 << 30;
  double4 *a = nullptr, *b = nullptr;
  double* o = nullptr;
  CHECK(hipMalloc(&a, total));
  CHECK(hipMalloc(&b, total));
  CHECK(hipMalloc(&o, 8));
  CHECK(hipMemset(a, 0, total));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const int gs[] = {1, 2, 8, 64, 256, 1024, 2048};
  for (int G : gs) {
    size_t per = (G <= 8) ? ((size_t)64 << 20) : total / G;
    per = per / 32 * 32;
    const size_t per4 = per / 32;
    hipLaunchKernelGGL(k_stream_read, dim3(G), dim3(512), 0, 0, a, per4, o);
    CHECK(hipEventRecord(e0));
    hipLaunchKernelGGL(k_stream_read, dim3(G), dim3(512), 0, 0, a, per4, o);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    std::printf("read G=%5d bytes/WG=%8.1f MB  %8.1f GB/s  (%.1f GB/s per workgroup)\n", G, per / 1e6,
                per * (double)G / (ms * 1e-3) / 1e9, per / (ms * 1e-3) / 1e9);
  }
  const size_t copy = (size_t)1 << 30, n4 = copy / 32;
  hipLaunchKernelGGL(k_plain_copy, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, 0, a, b, n4);
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(k_plain_copy, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, 0, a, b, n4);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  std::printf("copy %zu bytes: %.1f GB/s (read + write)\n", copy, 2.0 * copy / (ms * 1e-3) / 1e9);
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  CHECK(hipFree(o));
  return 0;
}
