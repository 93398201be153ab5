// Receiver sampling, adjoint sources, gradient accumulation and the FP64 local residual.
#include <algorithm>
#include <map>
#include <mutex>

#include "hbj_internal.h"

namespace {

// resid[s][r] = u[s][rec[r]] - d[s][r]
__global__ void k_gather_receivers(const double2* u, const int32_t* rec, int nrec, int npts, const double2* d,
                                   double2* resid, int nsrc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrec * nsrc) return;
  const int s = t / nrec, r = t - s * nrec;
  const double2 v = u[(size_t)s * npts + rec[r]];
  const double2 dd = d[t];
  resid[t] = mk(v.x - dd.x, v.y - dd.y);
}

// f_adj[s] = conj(P^T resid[s])  (f_adj must be zeroed; receivers are distinct nodes)
__global__ void k_spread_adjoint(const double2* resid, const int32_t* rec, int nrec, int npts, double2* f_adj,
                                 int nsrc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrec * nsrc) return;
  const int s = t / nrec, r = t - s * nrec;
  f_adj[(size_t)s * npts + rec[r]] = cconj(resid[t]);
}

// grad_p += sum_s -Re(conj(lambda) dA_pp/dm_p u) with lambda = conj(mu), i.e. -Re(mu dA u).
// dA_pp/dm_p = -k^2 - sum_{outer faces} (1/h^2) (i/h)/beta-^2 * k / (2 sqrt(m_p)).
__global__ void k_grad_accumulate(Geom g, const double* m, const double2* u, const double2* mu, int nsrc,
                                  double* grad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int npts = g.nx * g.ny;
  if (t >= npts) return;
  const int iy = t / g.nx, ix = t - iy * g.nx;
  const int nout = (ix == 0) + (ix == g.nx - 1) + (iy == 0) + (iy == g.ny - 1);
  double2 dA = mk(-g.k * g.k, 0.0);
  if (nout) {
    const double mp = m[t];
    const double alpha = g.k * sqrt(mp);
    const double2 bm = mk(1.0 / g.h, -0.5 * alpha);
    const double2 bm2 = cmul(bm, bm);
    const double2 drho = cdiv(mk(0.0, 1.0 / g.h), bm2);
    const double dalpha = g.k / (2.0 * sqrt(mp));
    const double sc = nout * dalpha / (g.h * g.h);
    dA.x -= sc * drho.x;
    dA.y -= sc * drho.y;
  }
  double acc = 0.0;
  for (int s = 0; s < nsrc; ++s) {
    const double2 a = cmul(mu[(size_t)s * npts + t], cmul(dA, u[(size_t)s * npts + t]));
    acc -= a.x;
  }
  grad[t] = acc;
}

// r = rhs - A_s x for every entry (complex128, matrix-free 5-point stencil + face diagonal)
// r = rhs - A_s x with A_s the 5-point operator, the face diagonal terms (diag) and, for the
// second-order transmission, the tangential couplings -s_{e,e+1} / h^2 between consecutive edge
// nodes of each interface face (band weights; zero for the first-order condition).
__global__ void k_local_residual(Geom g, const Entry* ent, const FaceTab* ft, const IfBand* band, const double2* diag,
                                 const double2* rhs64, const double2* x64, double2* r64) {
  const int slot = blockIdx.y;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= g.nloc) return;
  const int s = ent[slot].s;
  const double2* x = x64 + (size_t)slot * g.nloc;
  const int ly = l / g.snx, lx = l - ly * g.snx;
  double2 ax = cmul(diag[(size_t)s * g.nloc + l], x[l]);
  const double off = -1.0 / (g.h * g.h);
  double2 nb = mk(0.0, 0.0);
  if (lx > 0) nb = cadd(nb, x[l - 1]);
  if (lx < g.snx - 1) nb = cadd(nb, x[l + 1]);
  if (ly > 0) nb = cadd(nb, x[l - g.snx]);
  if (ly < g.sny - 1) nb = cadd(nb, x[l + g.snx]);
  ax.x += off * nb.x;
  ax.y += off * nb.y;
  const FaceTab F = ft[s];
  const bool on[4] = {lx == 0, lx == g.snx - 1, ly == 0, ly == g.sny - 1};
  for (int f = 0; f < 4; ++f) {
    if (!on[f] || F.in_off[f] < 0) continue;
    const int e = f < 2 ? ly : lx, len = f < 2 ? g.sny : g.snx, step = f < 2 ? g.snx : 1;
    const IfBand& B = band[F.in_off[f] + e];
    if (e > 0) cfma(ax, mk(off * B.t[0].x, off * B.t[0].y), x[l - step]);
    if (e < len - 1) cfma(ax, mk(off * B.t[1].x, off * B.t[1].y), x[l + step]);
  }
  const double2 b = rhs64[(size_t)slot * g.nloc + l];
  r64[(size_t)slot * g.nloc + l] = mk(b.x - ax.x, b.y - ax.y);
}

// Residual of the global discrete problem (Sec. 3, eq. (1)): r = f - A u with A the 5-point
// operator on the whole grid, whose outer faces carry the absorbing condition (ghost value
// rho_b u_p, rho_b = beta+/beta- with alpha_b = k sqrt(m_p)).  Workgroup (b, rhs) sums |r|^2 and
// |f|^2 over its share of the nodes (grid-stride) and writes the two sums to
// part[(rhs * nblk + b) * 2 + {0, 1}].
constexpr int kVrThreads = 256;
constexpr int kVrMaxBlocks = 1024;  // workgroups per right-hand side of k_volume_residual
__global__ void __launch_bounds__(kVrThreads) k_volume_residual(Geom g, const double* m, const double2* f,
                                                                const double2* u, int nblk, double* part) {
  const int rhs = blockIdx.y;
  const int npts = g.nx * g.ny;
  const double2* ur = u + (size_t)rhs * npts;
  const double2* fr = f + (size_t)rhs * npts;
  const double ih2 = 1.0 / (g.h * g.h);
  double rr = 0.0, ff = 0.0;
  for (int t = blockIdx.x * kVrThreads + threadIdx.x; t < npts; t += nblk * kVrThreads) {
    const int iy = t / g.nx, ix = t - iy * g.nx;
    const double2 up = ur[t];
    const int nout = (ix == 0) + (ix == g.nx - 1) + (iy == 0) + (iy == g.ny - 1);
    double2 nb = mk(0.0, 0.0);
    if (ix > 0) nb = cadd(nb, ur[t - 1]);
    if (ix < g.nx - 1) nb = cadd(nb, ur[t + 1]);
    if (iy > 0) nb = cadd(nb, ur[t - g.nx]);
    if (iy < g.ny - 1) nb = cadd(nb, ur[t + g.nx]);
    double2 d = mk(4.0 * ih2 - g.k * g.k * m[t], 0.0);
    if (nout) {
      const double alpha = g.k * sqrt(m[t]);
      const double2 rho = cdiv(mk(1.0 / g.h, 0.5 * alpha), mk(1.0 / g.h, -0.5 * alpha));
      d.x -= nout * rho.x * ih2;
      d.y -= nout * rho.y * ih2;
    }
    double2 au = cmul(d, up);
    au.x -= ih2 * nb.x;
    au.y -= ih2 * nb.y;
    const double2 fv = fr[t];
    const double rx = fv.x - au.x, ry = fv.y - au.y;
    rr += rx * rx + ry * ry;
    ff += fv.x * fv.x + fv.y * fv.y;
  }
  __shared__ double sr[kVrThreads], sf[kVrThreads];
  sr[threadIdx.x] = rr;
  sf[threadIdx.x] = ff;
  __syncthreads();
  for (int w = kVrThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sr[threadIdx.x] += sr[threadIdx.x + w];
      sf[threadIdx.x] += sf[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)rhs * nblk + blockIdx.x) * 2 + 0] = sr[0];
    part[((size_t)rhs * nblk + blockIdx.x) * 2 + 1] = sf[0];
  }
}

// Sums of the nblk partial pairs of right-hand side rhs = blockIdx.x (one workgroup per rhs); the
// result is valid in thread 0.
__device__ inline void sum_partial_pairs(const double* part, int nblk, double* rr_out, double* ff_out) {
  const int rhs = blockIdx.x;
  double rr = 0.0, ff = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kVrThreads) {
    rr += part[((size_t)rhs * nblk + b) * 2 + 0];
    ff += part[((size_t)rhs * nblk + b) * 2 + 1];
  }
  __shared__ double sr[kVrThreads], sf[kVrThreads];
  sr[threadIdx.x] = rr;
  sf[threadIdx.x] = ff;
  __syncthreads();
  for (int w = kVrThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sr[threadIdx.x] += sr[threadIdx.x + w];
      sf[threadIdx.x] += sf[threadIdx.x + w];
    }
    __syncthreads();
  }
  *rr_out = sr[0];
  *ff_out = sf[0];
}

// out[rhs * 2 + {0, 1}] = sums of the nblk partial pairs of rhs (one workgroup per rhs)
__global__ void __launch_bounds__(kVrThreads) k_volume_residual_sum(const double* part, int nblk, double* out) {
  double rr, ff;
  sum_partial_pairs(part, nblk, &rr, &ff);
  if (threadIdx.x == 0) {
    out[blockIdx.x * 2 + 0] = rr;
    out[blockIdx.x * 2 + 1] = ff;
  }
}

// relres[rhs] = sqrt(|r|^2 / |f|^2) from the partial pairs of rhs (sqrt(|r|^2) when f = 0), left on
// the device: the second stage of the allocation-free variant
__global__ void __launch_bounds__(kVrThreads) k_volume_residual_ratio(const double* part, int nblk,
                                                                     double* relres) {
  double rr, ff;
  sum_partial_pairs(part, nblk, &rr, &ff);
  if (threadIdx.x == 0) relres[blockIdx.x] = ff > 0.0 ? sqrt(rr / ff) : sqrt(rr);
}

// Scratch of the allocation-free volume residual: the partial pairs of every workgroup for at
// most HBJ_VR_NOALLOC_MAX_RHS right-hand sides (1 MiB).  Each device holds its own copy until the
// process ends.  Host code never passes this name to a kernel: it uses the device address that
// hipGetSymbolAddress returned for the device (volume_residual_scratch_init).
static __device__ __align__(256) double scratch[(size_t)HBJ_VR_NOALLOC_MAX_RHS * kVrMaxBlocks * 2];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;  // device ordinal -> address of that device's scratch

// ratio[e] = ||r_e|| / ||b_e|| for the local vectors of entry e (0 when b_e = 0): the relative
// residual of each refined local solve (one workgroup per entry)
__global__ void __launch_bounds__(kVrThreads) k_entry_ratio(const double2* r, const double2* b, int nloc,
                                                            double* ratio) {
  const size_t base = (size_t)blockIdx.x * nloc;
  double rr = 0.0, bb = 0.0;
  for (int l = threadIdx.x; l < nloc; l += kVrThreads) {
    const double2 rv = r[base + l], bv = b[base + l];
    rr += rv.x * rv.x + rv.y * rv.y;
    bb += bv.x * bv.x + bv.y * bv.y;
  }
  __shared__ double sr[kVrThreads], sb[kVrThreads];
  sr[threadIdx.x] = rr;
  sb[threadIdx.x] = bb;
  __syncthreads();
  for (int w = kVrThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sr[threadIdx.x] += sr[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) ratio[blockIdx.x] = sb[0] > 0.0 ? sqrt(sr[0] / sb[0]) : 0.0;
}

inline dim3 grid1(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_entry_ratio(const double2* r, const double2* b, int nloc, int nent, double* ratio, hipStream_t st) {
  if (nent <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_entry_ratio, dim3(nent), dim3(kVrThreads), 0, st, r, b, nloc, ratio);
  return hipGetLastError();
}

int volume_residual_blocks(const Geom& g) {
  const int npts = g.nx * g.ny;
  return std::max(1, std::min(kVrMaxBlocks, (npts + kVrThreads - 1) / kVrThreads));
}

hipError_t launch_volume_residual(const Geom& g, const double* m, const double2* f, const double2* u, int nrhs,
                                  double* part, double* sums, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  const int nblk = volume_residual_blocks(g);
  hipLaunchKernelGGL(k_volume_residual, dim3(nblk, nrhs), dim3(kVrThreads), 0, st, g, m, f, u, nblk, part);
  hipLaunchKernelGGL(k_volume_residual_sum, dim3(nrhs), dim3(kVrThreads), 0, st, part, nblk, sums);
  return hipGetLastError();
}

hipError_t volume_residual_scratch_init(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(dev)) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = static_cast<double*>(p);
  return hipSuccess;
}

hipError_t launch_volume_residual_noalloc(int dev, const Geom& g, const double* m, const double2* f,
                                          const double2* u, int nrhs, double* relres, hipStream_t st) {
  if (nrhs <= 0 || nrhs > HBJ_VR_NOALLOC_MAX_RHS) return hipErrorInvalidValue;
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) part = it->second;
  }
  if (!part) return hipErrorNotInitialized;
  const int nblk = volume_residual_blocks(g);
  hipLaunchKernelGGL(k_volume_residual, dim3(nblk, nrhs), dim3(kVrThreads), 0, st, g, m, f, u, nblk, part);
  hipLaunchKernelGGL(k_volume_residual_ratio, dim3(nrhs), dim3(kVrThreads), 0, st, part, nblk, relres);
  return hipGetLastError();
}

hipError_t launch_gather_receivers(const double2* u, const int32_t* rec, int nrec, int npts, const double2* d,
                                   double2* resid, int nsrc, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_receivers, grid1((size_t)nrec * nsrc), dim3(256), 0, st, u, rec, nrec, npts, d, resid,
                     nsrc);
  return hipGetLastError();
}

hipError_t launch_spread_adjoint(const double2* resid, const int32_t* rec, int nrec, int npts, double2* f_adj,
                                 int nsrc, hipStream_t st) {
  hipLaunchKernelGGL(k_spread_adjoint, grid1((size_t)nrec * nsrc), dim3(256), 0, st, resid, rec, nrec, npts, f_adj,
                     nsrc);
  return hipGetLastError();
}

hipError_t launch_grad_accumulate(const Geom& g, const double* m, const double2* u, const double2* mu, int nsrc,
                                  double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_accumulate, grid1((size_t)g.nx * g.ny), dim3(256), 0, st, g, m, u, mu, nsrc, grad);
  return hipGetLastError();
}

hipError_t launch_local_residual(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfBand* band,
                                 const double2* diag, const double2* rhs64, const double2* x64, double2* r64,
                                 hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_local_residual, dim3((g.nloc + 255) / 256, nent), dim3(256), 0, st, g, ent, ft, band, diag,
                     rhs64, x64, r64);
  return hipGetLastError();
}
