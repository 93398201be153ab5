// Receiver sampling, adjoint sources, gradient accumulation and the FP64 local residual.
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

inline dim3 grid1(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

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
