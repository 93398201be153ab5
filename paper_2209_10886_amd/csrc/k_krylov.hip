// Krylov-vector kernels for (F)GMRES on the interface system (complex128).
//
// Vectors come in column blocks [ncol][n] (one column per right-hand side).  Every
// reduction is deterministic: each workgroup sums a fixed chunk in a fixed order
// (per-thread strided sums, then a wavefront shuffle tree, then an LDS tree over the
// waves), and a second kernel adds the per-chunk partials in chunk order.
#include "hbj_internal.h"

namespace {

constexpr int RT = 256;  // threads per reduction workgroup

// Sum over the 64 lanes of a wavefront with DPP moves only (no LDS traffic): a running sum inside
// each row of 16 lanes (row_shr 1, 2, 4, 8), then rows 1 and 3 add the last lane of the row before
// (row_bcast:15) and rows 2 and 3 the last lane of row 1 (row_bcast:31).  Lane 63 ends with the sum.
template <int CTRL, int ROWS>
__device__ inline double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return v + __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline double wave_sum_last(double v) {
  v = dpp_add<0x111, 0xF>(v);  // row_shr:1
  v = dpp_add<0x112, 0xF>(v);  // row_shr:2
  v = dpp_add<0x114, 0xF>(v);  // row_shr:4
  v = dpp_add<0x118, 0xF>(v);  // row_shr:8
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

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
constexpr int VG = 8;
__global__ __launch_bounds__(RT) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_multidot(const double2* V, size_t vstride, int nvec, const double2* w,
                                                 int n, double2* partial, int nchunk) {
  const int chunk = blockIdx.x, i0 = blockIdx.y * VG, col = blockIdx.z;
  const int len = (n + nchunk - 1) / nchunk;
  const int q0 = chunk * len, q1 = min(n, q0 + len);
  const double2* ww = w + (size_t)col * n;
  double2 acc[VG];
#pragma unroll
  for (int v = 0; v < VG; ++v) acc[v] = mk(0.0, 0.0);
  // sub-blocks of 4 x RT entries; every load of a sub-block is issued before its products:
  // indices past the chunk or past the last vector are clamped (in bounds) and their
  // contributions are zeroed through w or dropped with the accumulator
  constexpr int U = 4;
  for (int qb = q0; qb < q1; qb += U * RT) {
    double2 wl[U];
    int qi[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int q = qb + threadIdx.x + k * RT;
      qi[k] = q < q1 ? q : q1 - 1;
      wl[k] = ww[qi[k]];
      if (q >= q1) wl[k] = mk(0.0, 0.0);
    }
    double2 vl[VG][U];
#pragma unroll
    for (int v = 0; v < VG; ++v) {
      const double2* vp = V + (size_t)min(i0 + v, nvec - 1) * vstride + (size_t)col * n;
#pragma unroll
      for (int k = 0; k < U; ++k) vl[v][k] = vp[qi[k]];
    }
#pragma unroll
    for (int v = 0; v < VG; ++v)
#pragma unroll
      for (int k = 0; k < U; ++k) cfma_conj(acc[v], vl[v][k], wl[k]);
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

// Fused Gram-Schmidt update: every workgroup first adds the dot-product partials of its column
// in chunk order (the same sums in every workgroup), workgroup 0 publishes h for the host, then
//   w[col][q] += alpha sum_i V_i[col][q] h_i
// and, if npart is given, the workgroup's partial sum of |w_new|^2 goes to npart[col][block].
constexpr int kFuseMax = 2048;  // nvec * nchunk held in LDS (32 KB)
__global__ __launch_bounds__(RT) void k_update_reduce(double2* w, const double2* V, size_t vstride, int nvec,
                                                      const double2* partial, int nchunk, double2* h_out,
                                                      size_t h_stride, double2 alpha, int n, double* npart) {
  const int col = blockIdx.y;
  __shared__ double2 sp[kFuseMax];
  __shared__ double2 hl[kFuseMax / 16];
  __shared__ double sn[RT / 64];
  const double2* pc = partial + (size_t)col * nvec * nchunk;
  const int np = nvec * nchunk;  // <= kFuseMax = 8 RT: one batch of loads per thread
  {
    double2 pv[kFuseMax / RT];
#pragma unroll
    for (int k = 0; k < kFuseMax / RT; ++k) {
      const int t = threadIdx.x + k * RT;
      pv[k] = pc[t < np ? t : np - 1];
    }
#pragma unroll
    for (int k = 0; k < kFuseMax / RT; ++k) sp[threadIdx.x + k * RT] = pv[k];  // entries >= np unused
  }
  __syncthreads();
  constexpr int UB = 8;  // basis vectors per batch of loads
  const int nv8 = (nvec + UB - 1) / UB * UB;
  if (threadIdx.x < nv8) {
    double2 h = mk(0.0, 0.0);
    if ((int)threadIdx.x < nvec) {
      for (int c = 0; c < nchunk; ++c) h = cadd(h, sp[threadIdx.x * nchunk + c]);
      if (blockIdx.x == 0) h_out[(size_t)col * h_stride + threadIdx.x] = h;
    }
    hl[threadIdx.x] = h;  // zero weights pad the last batch
  }
  __syncthreads();
  const int q = blockIdx.x * RT + threadIdx.x;
  double sq = 0.0;
  const size_t t = (size_t)col * n + (q < n ? q : n - 1);
  double2 acc = mk(0.0, 0.0);
  for (int i0 = 0; i0 < nv8; i0 += UB) {
    double2 vl[UB];
#pragma unroll
    for (int k = 0; k < UB; ++k) vl[k] = V[(size_t)min(i0 + k, nvec - 1) * vstride + t];
#pragma unroll
    for (int k = 0; k < UB; ++k) cfma(acc, vl[k], hl[i0 + k]);
  }
  if (q < n) {
    double2 r = w[t];
    cfma(r, alpha, acc);
    w[t] = r;
    sq = r.x * r.x + r.y * r.y;
  }
  if (npart) {
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sn[wid] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < RT / 64; ++k) t += sn[k];
      npart[(size_t)col * gridDim.x + blockIdx.x] = t;
    }
  }
}

// nrm[col] = sqrt(sum_b npart[col][b]) (fixed pairwise order), dst = src / nrm (0 if nrm = 0);
// workgroup 0 publishes nrm for the host
__global__ __launch_bounds__(RT) void k_scale_reduce(double2* dst, const double2* src, const double* npart,
                                                     int nblk, double* nrm_out, int n) {
  const int col = blockIdx.y;
  __shared__ double sp[RT];
  double pv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {  // clamped loads, all issued before use
    const int t = threadIdx.x + k * RT;
    pv[k] = npart[(size_t)col * nblk + (t < nblk ? t : nblk - 1)];
    if (t >= nblk) pv[k] = 0.0;
  }
  sp[threadIdx.x] = (pv[0] + pv[1]) + (pv[2] + pv[3]);
  __syncthreads();
  for (int half = RT / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half) sp[threadIdx.x] += sp[threadIdx.x + half];
    __syncthreads();
  }
  const double a = sqrt(sp[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) nrm_out[col] = a;
  const int q = blockIdx.x * RT + threadIdx.x;
  if (q < n) {
    const size_t t = (size_t)col * n + q;
    const double2 v = src[t];
    dst[t] = (a > 0.0) ? mk(v.x / a, v.y / a) : mk(0.0, 0.0);
  }
}

// ---------------------------------------------------------------------------------------------
// Gram-Schmidt with delayed reorthogonalisation (Bielich, Langou, Thomas, Swirydowicz, Yamazaki
// and Boman, 2022): Arnoldi step j receives x, the vector that went through one Gram-Schmidt pass
// at step j - 1, and w = (I - S) P^{-1} x.  One pass over the finished basis V_0..V_{nv-1}
// (nv = j) gives every inner product the step needs; one more pass finishes v_j (the second,
// delayed pass for x, with Pythagoras for its norm) and makes the next x from w.  The basis is
// read twice per step instead of four times.

// partial[(col * np + i) * nchunk + chunk], np = 2 nv + 3:
//   i < nv: V_i^H x;  nv + i: V_i^H w;  2 nv: x^H x;  2 nv + 1: x^H w;  2 nv + 2: w^H w.
// Grid (nchunk, max(1, ceil(nv / VG)), ncol); group 0 also sums the three products of x and w.
constexpr int VG2 = 4;  // basis vectors per workgroup (4: twice the workgroups of 8, 1% faster per solve at 1024^2)
template <int RT2, int U>  // threads, entries per thread and block of loads
__global__ __launch_bounds__(RT2) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_dots2(
    const double2* V, size_t vstride, int nv, const double2* x, const double2* w, int n, double2* partial,
    int nchunk) {
  const int chunk = blockIdx.x, i0 = blockIdx.y * VG2, col = blockIdx.z;
  const int len = (n + nchunk - 1) / nchunk;
  const int q0 = chunk * len, q1 = min(n, q0 + len);
  const double2* xx = x + (size_t)col * n;
  const double2* ww = w + (size_t)col * n;
  const bool g0 = blockIdx.y == 0;
  double2 aa[VG2], ab[VG2];
#pragma unroll
  for (int v = 0; v < VG2; ++v) aa[v] = ab[v] = mk(0.0, 0.0);
  double sxx = 0.0, sww = 0.0;
  double2 sxw = mk(0.0, 0.0);
  for (int qb = q0; qb < q1; qb += U * RT2) {
    // every load of the block is issued, with clamped (in-bounds) indices, before any is used;
    // entries past the chunk are zeroed afterwards, and with nv = 0 the basis loads read V_0
    // (products that are never stored)
    double2 xl[U], wl[U];
    int qi[U], vm = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int q = qb + threadIdx.x + k * RT2;
      vm |= (int)(q < q1) << k;
      qi[k] = q < q1 ? q : q1 - 1;
      xl[k] = xx[qi[k]];
      wl[k] = ww[qi[k]];
    }
    double2 vl[VG2][U];
#pragma unroll
    for (int v = 0; v < VG2; ++v) {
      const double2* vp = V + (size_t)max(0, min(i0 + v, nv - 1)) * vstride + (size_t)col * n;
#pragma unroll
      for (int k = 0; k < U; ++k) vl[v][k] = vp[qi[k]];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const bool in = (vm >> k) & 1;
      xl[k] = in ? xl[k] : mk(0.0, 0.0);
      wl[k] = in ? wl[k] : mk(0.0, 0.0);
    }
#pragma unroll
    for (int v = 0; v < VG2; ++v)
#pragma unroll
      for (int k = 0; k < U; ++k) {
        cfma_conj(aa[v], vl[v][k], xl[k]);
        cfma_conj(ab[v], vl[v][k], wl[k]);
      }
    if (g0) {
#pragma unroll
      for (int k = 0; k < U; ++k) {
        sxx += xl[k].x * xl[k].x + xl[k].y * xl[k].y;
        sww += wl[k].x * wl[k].x + wl[k].y * wl[k].y;
        cfma_conj(sxw, xl[k], wl[k]);
      }
    }
  }
  constexpr int NS = 2 * VG2 + 2;  // a, b, then (xx, ww) and xw
  __shared__ double2 sh[RT2 / 64][NS];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double2 vals[NS];
#pragma unroll
  for (int v = 0; v < VG2; ++v) {
    vals[v] = aa[v];
    vals[VG2 + v] = ab[v];
  }
  vals[2 * VG2] = mk(sxx, sww);
  vals[2 * VG2 + 1] = sxw;
  // wavefront sums with DPP moves (lane 63 holds them)
#pragma unroll
  for (int v = 0; v < NS; ++v) {
    vals[v].x = wave_sum_last(vals[v].x);
    vals[v].y = wave_sum_last(vals[v].y);
  }
  if (lane == 63)
#pragma unroll
    for (int v = 0; v < NS; ++v) sh[wid][v] = vals[v];
  __syncthreads();
  const int np = 2 * nv + 3;
  double2* pc = partial + (size_t)col * np * nchunk + chunk;
  if (threadIdx.x < NS) {
    double2 t = mk(0.0, 0.0);
    for (int q = 0; q < RT2 / 64; ++q) t = cadd(t, sh[q][threadIdx.x]);
    const int v = threadIdx.x;
    if (v < VG2) {
      if (i0 + v < nv) pc[(size_t)(i0 + v) * nchunk] = t;
    } else if (v < 2 * VG2) {
      if (i0 + v - VG2 < nv) pc[(size_t)(nv + i0 + v - VG2) * nchunk] = t;
    } else if (g0 && v == 2 * VG2) {
      pc[(size_t)(2 * nv) * nchunk] = mk(t.x, 0.0);
      pc[(size_t)(2 * nv + 2) * nchunk] = mk(t.y, 0.0);
    } else if (g0) {
      pc[(size_t)(2 * nv + 1) * nchunk] = t;
    }
  }
}

// Second pass of step j.  Every workgroup adds the partials of its column in chunk order (the same
// sums everywhere) and forms
//   a = V^H x,  nu = sqrt(x^H x - |a|^2),  v_j = (x - V a) / nu,
//   c_i = V_i^H w (i < j),  c_j = v_j^H w = (x^H w - a^H V^H w) / nu,  s = |w|,
//   x_next = (w - V c - v_j c_j) / s;
// v_j overwrites x in place and x_next goes to xn.  Workgroup 0 stores, per column, a (nv values)
// at hout[col * ld], c (nv + 1 values) at hout[(ncol + col) * ld] and (nu, s, |w|^2) as doubles at
// hout + 2 ncol ld + 2 col, for the host, which completes Hessenberg column j - 1 with them.
// publish_only: only the coefficients (the last step of a restart cycle, which needs a and nu).
constexpr int kDcgsMaxV = 256;
constexpr int kDcgsThreads = 256;  // threads per update workgroup, one position each (128 and 512 were slower)
constexpr int kDotsThreads = 256, kDotsBlock = 2;  // fastest of a sweep over 128-1024 threads, 2-4 entries
__global__ __launch_bounds__(kDcgsThreads) void k_dcgs_update(const double2* V, size_t vstride, int nv, double2* x,
                                                    double2* xn, const double2* w, const double2* partial,
                                                    int nchunk, double2* hout, int ld, int n, int publish_only) {
  const int col = blockIdx.y, ncol = gridDim.y;
  __shared__ double2 sp[kFuseMax];
  __shared__ double2 ca[kDcgsMaxV], cb[kDcgsMaxV];
  __shared__ double sc[8];
  __shared__ double2 scj[1];
  const int np = 2 * nv + 3;
  const double2* pc = partial + (size_t)col * np * nchunk;
  const int nt = np * nchunk;  // <= kFuseMax
  {
    double2 pv[kFuseMax / kDcgsThreads];
#pragma unroll
    for (int k = 0; k < kFuseMax / kDcgsThreads; ++k) {
      const int t = threadIdx.x + k * kDcgsThreads;
      pv[k] = pc[t < nt ? t : nt - 1];
    }
#pragma unroll
    for (int k = 0; k < kFuseMax / kDcgsThreads; ++k) sp[threadIdx.x + k * kDcgsThreads] = pv[k];
  }
  __syncthreads();
  const int nv8 = (nv + 7) / 8 * 8;
  constexpr int kRows = (2 * kDcgsMaxV + 3 + kDcgsThreads - 1) / kDcgsThreads;  // rows of sums per thread
  double2 tsum[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int i = threadIdx.x + r * kDcgsThreads;
    tsum[r] = mk(0.0, 0.0);
    if (i < np)
      for (int c = 0; c < nchunk; ++c) tsum[r] = cadd(tsum[r], sp[i * nchunk + c]);
  }
  __syncthreads();  // sp is reused below for the sums
#pragma unroll
  for (int r = 0; r < kRows; ++r)
    if ((int)threadIdx.x + r * kDcgsThreads < np) sp[threadIdx.x + r * kDcgsThreads] = tsum[r];
  __syncthreads();
  for (int i = threadIdx.x; i < nv8; i += kDcgsThreads) {  // zero weights pad the last batch
    ca[i] = i < nv ? sp[i] : mk(0.0, 0.0);
    cb[i] = i < nv ? sp[nv + i] : mk(0.0, 0.0);
  }
  if (threadIdx.x < 64) {
    // |a|^2 and a^H b over wavefront 0: strided per-lane sums, then a DPP sum (fixed order)
    double na = 0.0;
    double2 ab = mk(0.0, 0.0);
    for (int i = threadIdx.x; i < nv; i += 64) {
      const double2 a = sp[i];
      na += a.x * a.x + a.y * a.y;
      cfma_conj(ab, a, sp[nv + i]);
    }
    na = wave_sum_last(na);  // DPP sums: lane 63 holds them
    ab.x = wave_sum_last(ab.x);
    ab.y = wave_sum_last(ab.y);
    if (threadIdx.x == 63) {
      const double xx = sp[2 * nv].x, ww = sp[2 * nv + 2].x;
      const double2 xw = sp[2 * nv + 1];
      const double nu2 = xx - na;
      const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
      const double s = ww > 0.0 ? sqrt(ww) : 0.0;
      sc[0] = nu;
      sc[1] = s;
      sc[2] = ww;
      sc[3] = nu > 0.0 ? 1.0 / nu : 0.0;
      sc[4] = s > 0.0 ? 1.0 / s : 0.0;
      scj[0] = nu > 0.0 ? mk((xw.x - ab.x) / nu, (xw.y - ab.y) / nu) : mk(0.0, 0.0);
    }
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i <= nv; i += kDcgsThreads) {
      if (i < nv) hout[(size_t)col * ld + i] = ca[i];
      hout[((size_t)ncol + col) * ld + i] = i < nv ? cb[i] : scj[0];
    }
    if (threadIdx.x == 0) {
      double* hs = (double*)(hout + 2 * (size_t)ncol * ld) + 4 * (size_t)col;
      hs[0] = sc[0];
      hs[1] = sc[1];
      hs[2] = sc[2];
      hs[3] = 0.0;
    }
  }
  if (publish_only) return;
  const int q = blockIdx.x * kDcgsThreads + threadIdx.x;
  const size_t t = (size_t)col * n + (q < n ? q : n - 1);
  const double2 xv = x[t], wv = w[t];
  double2 accA = mk(0.0, 0.0), accB = mk(0.0, 0.0);
  constexpr int UB = 8;  // basis vectors per batch of loads
  for (int i0 = 0; i0 < nv8; i0 += UB) {
    double2 vl[UB];
#pragma unroll
    for (int k = 0; k < UB; ++k) vl[k] = V[(size_t)min(i0 + k, nv - 1) * vstride + t];
#pragma unroll
    for (int k = 0; k < UB; ++k) {
      cfma(accA, vl[k], ca[i0 + k]);
      cfma(accB, vl[k], cb[i0 + k]);
    }
  }
  if (q < n) {
    const double inu = sc[3], is = sc[4];
    const double2 v = mk((xv.x - accA.x) * inu, (xv.y - accA.y) * inu);
    double2 r = mk(wv.x - accB.x, wv.y - accB.y);
    const double2 cj = scj[0];
    r.x -= v.x * cj.x - v.y * cj.y;
    r.y -= v.x * cj.y + v.y * cj.x;
    x[t] = v;
    xn[t] = mk(r.x * is, r.y * is);
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

__global__ void k_zero_bytes(uint32_t* dst, size_t nwords) {  // grid-stride: any size
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nwords; t += (size_t)gridDim.x * blockDim.x)
    dst[t] = 0u;
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
  if (nchunk < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_multidot, dim3(nchunk, (nvec + VG - 1) / VG, ncol), dim3(RT), 0, st, V, vstride, nvec, w, n,
                     partial, nchunk);
  return hipGetLastError();
}

bool krylov_fusable(int nvec, int nchunk, int n) {
  return nvec * nchunk <= kFuseMax && nvec + 8 <= kFuseMax / 16 && (n + RT - 1) / RT <= 1024;
}

hipError_t launch_update_reduce(double2* w, const double2* V, size_t vstride, int nvec, const double2* partial,
                                int nchunk, double2* h_out, size_t h_stride, double2 alpha, int n, int ncol,
                                double* npart, hipStream_t st) {
  if (!krylov_fusable(nvec, nchunk, n)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_update_reduce, dim3((n + RT - 1) / RT, ncol), dim3(RT), 0, st, w, V, vstride, nvec, partial,
                     nchunk, h_out, h_stride, alpha, n, npart);
  return hipGetLastError();
}

hipError_t launch_scale_reduce(double2* dst, const double2* src, const double* npart, double* nrm_out, int n, int ncol,
                               hipStream_t st) {
  const int nblk = (n + RT - 1) / RT;
  if (nblk > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scale_reduce, dim3(nblk, ncol), dim3(RT), 0, st, dst, src, npart, nblk, nrm_out, n);
  return hipGetLastError();
}

bool dcgs_fits(int m, int nchunk) { return m + 1 <= kDcgsMaxV && (2 * m + 3) * nchunk <= kFuseMax; }

hipError_t launch_dots2(const double2* V, size_t vstride, int nv, const double2* x, const double2* w, int n, int ncol,
                        double2* partial, int nchunk, hipStream_t st) {
  if (nchunk < 1 || (2 * nv + 3) * nchunk > kFuseMax || nv + 1 > kDcgsMaxV) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_dots2<kDotsThreads, kDotsBlock>), dim3(nchunk, std::max(1, (nv + VG2 - 1) / VG2), ncol),
                     dim3(kDotsThreads), 0, st, V, vstride, nv, x, w, n, partial, nchunk);
  return hipGetLastError();
}

hipError_t launch_dcgs_update(const double2* V, size_t vstride, int nv, double2* x, double2* xn, const double2* w,
                              const double2* partial, int nchunk, double2* hout, int ld, int n, int ncol,
                              bool publish_only, hipStream_t st) {
  if (nchunk < 1 || (2 * nv + 3) * nchunk > kFuseMax || nv + 1 > kDcgsMaxV || nv + 1 > ld) return hipErrorInvalidValue;
  const int nblk = publish_only ? 1 : (n + kDcgsThreads - 1) / kDcgsThreads;
  hipLaunchKernelGGL(k_dcgs_update, dim3(nblk, ncol), dim3(kDcgsThreads), 0, st, V, vstride, nv, x, xn, w, partial, nchunk, hout,
                     ld, n, publish_only ? 1 : 0);
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
  const size_t nb = std::min<size_t>((nw + 255) / 256, (size_t)1 << 16);
  hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)nb), dim3(256), 0, st, (uint32_t*)dst, nw);
  return hipGetLastError();
}

hipError_t launch_add_ranges(double2* y, const double2* x, const int32_t* ranges, int nranges, int nif, int ncol,
                             hipStream_t st) {
  if (nranges == 0 || nif == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_ranges, grid1((size_t)nif * ncol), dim3(256), 0, st, y, x, ranges, nranges, nif, ncol);
  return hipGetLastError();
}
