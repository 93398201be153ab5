// Assembly of the local Helmholtz operators (paper Sec. 3, eq. (2)).
//
// Every subdomain matrix A_i is the 5-point operator on the subdomain's nodes,
//   (A u)_p = (4 u_p - sum_{nbrs in subdomain} u_q) / h^2 - k^2 m_p u_p - sum_{faces of p} rho_f u_p / h^2,
// where each face crossing the subdomain boundary carries the Robin template
// (u_q - u_p)/h - i alpha (u_p + u_q)/2 = g.  Eliminating the ghost u_q gives
// the -rho_f/h^2 diagonal term (rho = beta+/beta-, beta+- = 1/h +- i alpha/2) and
// the right-hand-side injection g/(beta- h^2).  alpha = k sqrt(m_p) on outer faces
// and k sqrt((m_p + m_q)/2) on interfaces (equal on both sides of the face).
#include "hbj_internal.h"

namespace {

__device__ inline void face_coeffs(double alpha, double h, double2& rho, double2& sigma, double2& inj) {
  const double2 bm = mk(1.0 / h, -0.5 * alpha);
  const double2 bp = mk(1.0 / h, 0.5 * alpha);
  rho = cdiv(bp, bm);
  sigma = cdiv(mk(0.0, 2.0 * alpha), mk(h * bm.x, h * bm.y));
  inj = cdiv(mk(1.0, 0.0), mk(bm.x * h * h, bm.y * h * h));
}

__global__ void k_check_medium(const double* c, int n, int* bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double v = c[i];
    if (!(v > 0.0) || !isfinite(v)) atomicAdd(bad, 1);
  }
}

__global__ void k_c_to_m(const double* c, double* m, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) m[i] = 1.0 / (c[i] * c[i]);
}

// pos_tab[q] = (subdomain, face, entry along the face, unused) of the receiver of position q
__global__ void k_if_coef(Geom g, const double* m, const int32_t* pos_tab, IfCoef* coef) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.nif) return;
  const int s = pos_tab[4 * q], f = pos_tab[4 * q + 1], e = pos_tab[4 * q + 2];
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
  int px, py, qx, qy;
  if (f == FACE_W) { px = x0; py = y0 + e; qx = px - 1; qy = py; }
  else if (f == FACE_E) { px = x0 + g.snx - 1; py = y0 + e; qx = px + 1; qy = py; }
  else if (f == FACE_S) { px = x0 + e; py = y0; qx = px; qy = py - 1; }
  else { px = x0 + e; py = y0 + g.sny - 1; qx = px; qy = py + 1; }
  const double mp = m[py * g.nx + px], mq = m[qy * g.nx + qx];
  const double alpha = g.k * sqrt(0.5 * (mp + mq));
  IfCoef c;
  face_coeffs(alpha, g.h, c.rho, c.sigma, c.inj);
  coef[q] = c;
}

// diag[s][l]: diagonal of A_s including every face term
__global__ void k_local_diag(Geom g, const double* m, const FaceTab* ft, const IfCoef* coef, double2* diag) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nsub = g.n1 * g.n2;
  if (t >= (size_t)nsub * g.nloc) return;
  const int s = (int)(t / g.nloc), l = (int)(t % g.nloc);
  const int ly = l / g.snx, lx = l - ly * g.snx;
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
  const double mp = m[(y0 + ly) * g.nx + x0 + lx];
  const double ih2 = 1.0 / (g.h * g.h);
  double2 d = mk(4.0 * ih2 - g.k * g.k * mp, 0.0);
  const FaceTab F = ft[s];
  const bool on[4] = {lx == 0, lx == g.snx - 1, ly == 0, ly == g.sny - 1};
  for (int f = 0; f < 4; ++f) {
    if (!on[f]) continue;
    double2 rho;
    if (F.in_off[f] >= 0) {
      rho = coef[F.in_off[f] + (f < 2 ? ly : lx)].rho;
    } else {
      double2 sg, ij;
      face_coeffs(g.k * sqrt(mp), g.h, rho, sg, ij);
    }
    d.x -= rho.x * ih2;
    d.y -= rho.y * ih2;
  }
  diag[t] = d;
}

// LAPACK band storage, column-major: A(i, j) at ab[j * ldab + kv + i - j]; rows [0, kl) are
// workspace for the fill of partial pivoting and start at zero.
__global__ void k_band_assemble(Geom g, const double2* diag, double2* ab, int nsub) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)g.nloc * g.ldab;
  if (t >= per * nsub) return;
  const int s = (int)(t / per);
  const size_t rem = t - (size_t)s * per;
  const int j = (int)(rem / g.ldab), r = (int)(rem % g.ldab);
  const int i = r - g.kv + j;  // row of A
  const double off = -1.0 / (g.h * g.h);
  double2 v = mk(0.0, 0.0);
  if (i >= 0 && i < g.nloc) {
    const int d = i - j;
    if (d == 0) v = diag[(size_t)s * g.nloc + j];
    else if (d == 1 && (j % g.snx) != g.snx - 1) v = mk(off, 0.0);
    else if (d == -1 && (j % g.snx) != 0) v = mk(off, 0.0);
    else if (d == g.snx || d == -g.snx) v = mk(off, 0.0);
  }
  ab[t] = v;
}

}  // namespace

hipError_t launch_check_medium(const double* c, int n, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_check_medium, dim3((n + 255) / 256), dim3(256), 0, st, c, n, bad);
  return hipGetLastError();
}

hipError_t launch_c_to_m(const double* c, double* m, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_c_to_m, dim3((n + 255) / 256), dim3(256), 0, st, c, m, n);
  return hipGetLastError();
}

hipError_t launch_if_coef(const Geom& g, const double* m, const int32_t* pos_tab, IfCoef* coef, hipStream_t st) {
  if (g.nif == 0) return hipSuccess;
  hipLaunchKernelGGL(k_if_coef, dim3((g.nif + 255) / 256), dim3(256), 0, st, g, m, pos_tab, coef);
  return hipGetLastError();
}

hipError_t launch_local_diag(const Geom& g, const double* m, const FaceTab* ft, const IfCoef* coef, double2* diag,
                             hipStream_t st) {
  const size_t n = (size_t)g.n1 * g.n2 * g.nloc;
  hipLaunchKernelGGL(k_local_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, m, ft, coef, diag);
  return hipGetLastError();
}

hipError_t launch_band_assemble(const Geom& g, const double2* diag, double2* ab, int nsub, hipStream_t st) {
  const size_t n = (size_t)nsub * g.nloc * g.ldab;
  hipLaunchKernelGGL(k_band_assemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, diag, ab, nsub);
  return hipGetLastError();
}
