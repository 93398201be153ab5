// HBM calibration probe (diagnostic program, not part of libhbj).
//
//  1. streaming reads: G workgroups each read their own contiguous chunk (8 independent 32-byte
//     loads in flight per thread); prints aggregate and per-workgroup GB/s for G = 1 .. 2048;
//  2. a plain copy of 1 GiB (the reference kernel whose FETCH_SIZE / WRITE_SIZE counters calibrate
//     the counter-based traffic figures of the solver kernels);
//  3. short launches: one launch reads S bytes (4 .. 212 MB) with G workgroups, timed from the
//     launch's own start and end events and averaged over 16 launches; "cold" launches each read a
//     different slice of a 2 GiB buffer (nothing left in the last-level cache), "warm" launches
//     re-read one slice.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

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
  // 3. short launches
  const double sizes_mb[] = {4.0, 12.5, 25.0, 50.0, 100.0, 212.0};
  const int wgs[] = {256, 512, 1024, 2048};
  constexpr int kReps = 16;
  hipEvent_t s0[kReps], s1[kReps];
  for (int r = 0; r < kReps; ++r) {
    CHECK(hipEventCreate(&s0[r]));
    CHECK(hipEventCreate(&s1[r]));
  }
  for (double mb : sizes_mb) {
    for (int G : wgs) {
      const size_t per4 = (size_t)(mb * 1e6 / 32.0) / G;  // double4 per workgroup
      const size_t slice4 = per4 * G;
      const size_t nslice = (total / 32) / slice4;  // disjoint slices in the 2 GiB buffer
      if (per4 == 0 || nslice < 2) continue;
      for (int warm = 0; warm < 2; ++warm) {
        hipLaunchKernelGGL(k_stream_read, dim3(G), dim3(512), 0, 0, a, per4, o);
        for (int r = 0; r < kReps; ++r) {
          const double4* src = a + (warm ? 0 : ((size_t)(r + 1) % nslice) * slice4);
          hipExtLaunchKernelGGL(k_stream_read, dim3(G), dim3(512), 0, 0, s0[r], s1[r], 0, src, per4, o);
        }
        CHECK(hipGetLastError());
        CHECK(hipDeviceSynchronize());
        double sum = 0;
        for (int r = 0; r < kReps; ++r) {
          float ms = 0;
          CHECK(hipEventElapsedTime(&ms, s0[r], s1[r]));
          sum += ms;
        }
        const double us = sum / kReps * 1e3;
        std::printf("short %s S=%6.1f MB G=%5d  %7.2f us  %8.1f GB/s\n", warm ? "warm" : "cold",
                    slice4 * 32.0 / 1e6, G, us, slice4 * 32.0 / (us * 1e-6) / 1e9);
      }
    }
  }
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  CHECK(hipFree(o));
  return 0;
}
