// Krylov-vector kernels for (F)GMRES on the interface system (complex128).
//
// Vectors come in column blocks [ncol][n] (one column per right-hand side).  Every
// reduction is deterministic: each workgroup sums a fixed chunk in a fixed order
// (per-thread strided sums, then a wavefront shuffle tree, then an LDS tree over the
// waves), and a second kernel adds the per-chunk partials in chunk order.
#include "hbj_internal.h"

namespace {

constexpr int RT = 256;  // threads per reduction workgroup

__device__ inline double2 shfl_down2(double2 v, int off) {
  v.x = __shfl_down(v.x, off);
  v.y = __shfl_down(v.y, off);
  return v;
}

__device__ inline double2 block_sum(double2 v, double2* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    const double2 o = shfl_down2(v, off);
    v.x += o.x;
    v.y += o.y;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double2 s = mk(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { s.x += sh[w].x; s.y += sh[w].y; }
  return s;
}

// partial[(col * nvec + i) * nchunk + chunk] = sum_{q in chunk} conj(V_i[col][q]) w[col][q].
// One workgroup per (chunk, group of VG basis vectors, column): the chunk of w is read once per
// group, the VG dot products accumulate in registers and meet in one block reduction.
constexpr int MD_PER_THREAD = 4;  // chunk = 1024 elements
constexpr int VG = 8;
__global__ __launch_bounds__(RT) void k_multidot(const double2* V, size_t vstride, int nvec, const double2* w,
                                                 int n, double2* partial, int nchunk) {
  const int chunk = blockIdx.x, i0 = blockIdx.y * VG, col = blockIdx.z;
  const int len = (n + nchunk - 1) / nchunk;
  const int q0 = chunk * len, q1 = min(n, q0 + len);
  const double2* ww = w + (size_t)col * n;
  double2 wl[MD_PER_THREAD];
#pragma unroll
  for (int k = 0; k < MD_PER_THREAD; ++k) {
    const int q = q0 + threadIdx.x + k * RT;
    wl[k] = (q < q1) ? ww[q] : mk(0.0, 0.0);
  }
  double2 acc[VG];
#pragma unroll
  for (int v = 0; v < VG; ++v) {
    acc[v] = mk(0.0, 0.0);
    if (i0 + v < nvec) {
      const double2* vp = V + (size_t)(i0 + v) * vstride + (size_t)col * n;
#pragma unroll
      for (int k = 0; k < MD_PER_THREAD; ++k) {
        const int q = q0 + threadIdx.x + k * RT;
        if (q < q1) cfma_conj(acc[v], vp[q], wl[k]);
      }
    }
  }
  __shared__ double2 sh[RT / 64][VG];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < VG; ++v) {
    double2 a = acc[v];
    for (int off = 32; off > 0; off >>= 1) {
      const double2 o = shfl_down2(a, off);
      a.x += o.x;
      a.y += o.y;
    }
    if (lane == 0) sh[wid][v] = a;
  }
  __syncthreads();
  if (threadIdx.x < VG && i0 + (int)threadIdx.x < nvec) {
    double2 t = mk(0.0, 0.0);
    for (int q = 0; q < RT / 64; ++q) t = cadd(t, sh[q][threadIdx.x]);
    partial[((size_t)col * nvec + i0 + threadIdx.x) * nchunk + chunk] = t;
  }
}

__global__ void k_reduce_partials(const double2* partial, int nvec, int ncol, int nchunk, double2* out,
                                  size_t out_stride, double2 scale) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nvec * ncol) return;
  const int col = t / nvec, i = t - col * nvec;
  const double2* p = partial + (size_t)t * nchunk;
  double2 s = mk(0.0, 0.0);
  for (int c = 0; c < nchunk; ++c) { s.x += p[c].x; s.y += p[c].y; }
  out[(size_t)col * out_stride + i] = cmul(s, scale);
}

// w[col][q] += alpha * sum_i V_i[col][q] h[col * h_stride + i]
__global__ void k_update(double2* w, const double2* V, size_t vstride, int nvec, const double2* h, size_t h_stride,
                         double2 alpha, int n, int ncol) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * ncol) return;
  const int col = (int)(t / n), q = (int)(t - (size_t)col * n);
  double2 acc = mk(0.0, 0.0);
  const double2* hc = h + (size_t)col * h_stride;
  for (int i = 0; i < nvec; ++i) cfma(acc, V[(size_t)i * vstride + t], hc[i]);
  double2 r = w[t];
  cfma(r, alpha, acc);
  w[t] = r;
}

__global__ __launch_bounds__(RT) void k_norm_partial(const double2* w, int n, double* partial, int nchunk) {
  const int chunk = blockIdx.x, col = blockIdx.y;
  const int len = (n + nchunk - 1) / nchunk;
  const int q0 = chunk * len, q1 = min(n, q0 + len);
  const double2* ww = w + (size_t)col * n;
  double2 acc = mk(0.0, 0.0);
  for (int q = q0 + threadIdx.x; q < q1; q += RT) acc.x = fma(ww[q].x, ww[q].x, fma(ww[q].y, ww[q].y, acc.x));
  __shared__ double2 sh[RT / 64];
  const double2 s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[(size_t)col * nchunk + chunk] = s.x;
}

__global__ void k_reduce_norms(const double* partial, int ncol, int nchunk, double* out) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[(size_t)col * nchunk + c];
  out[col] = sqrt(s);
}

__global__ void k_scale_by_inv(double2* dst, const double2* src, const double* nrm, int n, int ncol) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * ncol) return;
  const int col = (int)(t / n);
  const double a = nrm[col];
  const double2 v = src[t];
  dst[t] = (a > 0.0) ? mk(v.x / a, v.y / a) : mk(0.0, 0.0);
}

__global__ void k_axpby(double2* y, const double2* x, double2 a, double2 b, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double2 r = cmul(b, y[t]);
  cfma(r, a, x[t]);
  y[t] = r;
}

__global__ void k_copy(double2* dst, const double2* src, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

__global__ void k_zero_bytes(uint32_t* dst, size_t nwords) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nwords) dst[t] = 0u;
}

// y[col][q] += x[col][q] for q in any of the [start, end) ranges
__global__ void k_add_ranges(double2* y, const double2* x, const int32_t* ranges, int nranges, int nif, int ncol) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nif * ncol) return;
  const int q = (int)(t % nif);
  for (int r = 0; r < nranges; ++r) {
    if (q >= ranges[2 * r] && q < ranges[2 * r + 1]) {
      y[t] = cadd(y[t], x[t]);
      return;
    }
  }
}

inline dim3 grid1(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_multidot(const double2* V, size_t vstride, int nvec, const double2* w, int n, int ncol,
                           double2* partial, int nchunk, hipStream_t st) {
  if ((size_t)nchunk * RT * MD_PER_THREAD < (size_t)n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_multidot, dim3(nchunk, (nvec + VG - 1) / VG, ncol), dim3(RT), 0, st, V, vstride, nvec, w, n,
                     partial, nchunk);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double2* partial, int nvec, int ncol, int nchunk, double2* out,
                                  size_t out_stride, double2 scale, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, grid1((size_t)nvec * ncol), dim3(256), 0, st, partial, nvec, ncol, nchunk,
                     out, out_stride, scale);
  return hipGetLastError();
}

hipError_t launch_update(double2* w, const double2* V, size_t vstride, int nvec, const double2* h, size_t h_stride,
                         double2 alpha, int n, int ncol, hipStream_t st) {
  hipLaunchKernelGGL(k_update, grid1((size_t)n * ncol), dim3(256), 0, st, w, V, vstride, nvec, h, h_stride, alpha, n,
                     ncol);
  return hipGetLastError();
}

hipError_t launch_norms(const double2* w, int n, int ncol, double* partial, int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_partial, dim3(nchunk, ncol), dim3(RT), 0, st, w, n, partial, nchunk);
  return hipGetLastError();
}

hipError_t launch_reduce_norms(const double* partial, int ncol, int nchunk, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_norms, grid1(ncol), dim3(256), 0, st, partial, ncol, nchunk, out);
  return hipGetLastError();
}

hipError_t launch_scale_by_inv(double2* dst, const double2* src, const double* nrm, int n, int ncol, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_by_inv, grid1((size_t)n * ncol), dim3(256), 0, st, dst, src, nrm, n, ncol);
  return hipGetLastError();
}

hipError_t launch_axpby(double2* y, const double2* x, double2 a, double2 b, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, grid1(n), dim3(256), 0, st, y, x, a, b, n);
  return hipGetLastError();
}

hipError_t launch_copy(double2* dst, const double2* src, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, grid1(n), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const size_t nw = bytes / 4;
  hipLaunchKernelGGL(k_zero_bytes, grid1(nw), dim3(256), 0, st, (uint32_t*)dst, nw);
  return hipGetLastError();
}

hipError_t launch_add_ranges(double2* y, const double2* x, const int32_t* ranges, int nranges, int nif, int ncol,
                             hipStream_t st) {
  if (nranges == 0 || nif == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_ranges, grid1((size_t)nif * ncol), dim3(256), 0, st, y, x, ranges, nranges, nif, ncol);
  return hipGetLastError();
}
