// Assembly of the local Helmholtz operators (paper Sec. 3, eq. (2)).
//
// Every subdomain matrix A_i is the 5-point operator on the subdomain's nodes,
//   (A u)_p = (4 u_p - sum_{nbrs in subdomain} u_q) / h^2 - k^2 m_p u_p - sum_{faces of p} rho_f u_p / h^2,
// where each face crossing the subdomain boundary carries the Robin template
// (u_q - u_p)/h - i alpha (u_p + u_q)/2 = g.  Eliminating the ghost u_q gives
// the -rho_f/h^2 diagonal term (rho = beta+/beta-, beta+- = 1/h +- i alpha/2) and
// the right-hand-side injection g/(beta- h^2).  alpha = k sqrt(m_p) on outer faces
// and k sqrt((m_p + m_q)/2) on interfaces (equal on both sides of the face).
//
// Second-order transmission (interface faces only; the outer faces keep the absorbing condition):
// d_n u - i alpha a u - (i b / alpha) d_tt u = g, with the face template
//   (u_q - u_p)/h - i alpha a (u_p + u_q)/2 - beta-_e (C u_p)_e = g_e,
// beta+- from the impedance alpha a, C the symmetric tangential operator along the face (edge
// weights s_{e,e+1} = (kappa_e + kappa_{e+1}) / (2 h^2), kappa = (i b / alpha) / beta-, Neumann
// closure at the face ends).  The ghost is u_q = (g + beta+ u_p)/beta- + (C u_p)_e: the row of p
// gains -(C u_p)_e / h^2 (symmetric), and the datum sent back across the face is
// -R g - Sigma u along the face with M = B+ + B- C, R = M B-^{-1}, Sigma = M B-^{-1} M - B-.
#include "hbj_internal.h"

namespace {

// beta+- = 1/h +- i alpha / 2 for a complex impedance alpha
__device__ inline void face_coeffs_c(double2 alpha, double h, double2& bm, double2& bp, double2& rho, double2& sigma,
                                     double2& inj) {
  bm = mk(1.0 / h + 0.5 * alpha.y, -0.5 * alpha.x);
  bp = mk(1.0 / h - 0.5 * alpha.y, 0.5 * alpha.x);
  rho = cdiv(bp, bm);
  sigma = cdiv(mk(-2.0 * alpha.y, 2.0 * alpha.x), mk(h * bm.x, h * bm.y));
  inj = cdiv(mk(1.0, 0.0), mk(bm.x * h * h, bm.y * h * h));
}

__device__ inline void face_coeffs(double alpha, double h, double2& rho, double2& sigma, double2& inj) {
  double2 bm, bp;
  face_coeffs_c(mk(alpha, 0.0), h, bm, bp, rho, sigma, inj);
}

// physical impedance k sqrt((m_p + m_q)/2) at entry e of face f of subdomain s
__device__ inline double if_alpha(const Geom& g, const double* m, int s, int f, int e) {
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
  int px, py, qx, qy;
  if (f == FACE_W) { px = x0; py = y0 + e; qx = px - 1; qy = py; }
  else if (f == FACE_E) { px = x0 + g.snx - 1; py = y0 + e; qx = px + 1; qy = py; }
  else if (f == FACE_S) { px = x0 + e; py = y0; qx = px; qy = py - 1; }
  else { px = x0 + e; py = y0 + g.sny - 1; qx = px; qy = py + 1; }
  return g.k * sqrt(0.5 * (m[py * g.nx + px] + m[qy * g.nx + qx]));
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
__global__ void k_if_coef(Geom g, const double* m, const int32_t* pos_tab, double2 ta, IfCoef* coef) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.nif) return;
  const int s = pos_tab[4 * q], f = pos_tab[4 * q + 1], e = pos_tab[4 * q + 2];
  const double alpha = if_alpha(g, m, s, f, e);
  IfCoef c;
  double2 bm, bp;
  face_coeffs_c(mk(ta.x * alpha, ta.y * alpha), g.h, bm, bp, c.rho, c.sigma, c.inj);
  coef[q] = c;
}

// R and Sigma rows and the tangential edge weights of every interface position (see the file
// header); positions e-2 .. e+2 of the same face are consecutive interface positions q-2 .. q+2.
__global__ void k_if_band(Geom g, const double* m, const int32_t* pos_tab, int order, double2 ta, double2 tb,
                          const IfCoef* coef, IfBand* band) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.nif) return;
  IfBand B;
  for (int d = 0; d < 3; ++d) B.r[d] = mk(0.0, 0.0);
  for (int d = 0; d < 5; ++d) B.sg[d] = mk(0.0, 0.0);
  B.t[0] = B.t[1] = mk(0.0, 0.0);
  if (order == 1) {
    B.r[1] = coef[q].rho;
    B.sg[2] = coef[q].sigma;
    band[q] = B;
    return;
  }
  const int s = pos_tab[4 * q], f = pos_tab[4 * q + 1], e = pos_tab[4 * q + 2];
  const int len = f < 2 ? g.sny : g.snx;
  const double ih2 = 1.0 / (g.h * g.h);
  // window x = e - 2 .. e + 2 (index 0 .. 4)
  double2 bm[5], bp[5], kap[5];
  bool in[5];
  for (int c = 0; c < 5; ++c) {
    const int x = e + c - 2;
    in[c] = x >= 0 && x < len;
    bm[c] = bp[c] = kap[c] = mk(0.0, 0.0);
    if (!in[c]) continue;
    const double alpha = if_alpha(g, m, s, f, x);
    double2 rho, sig, inj;
    face_coeffs_c(mk(ta.x * alpha, ta.y * alpha), g.h, bm[c], bp[c], rho, sig, inj);
    kap[c] = cdiv(mk(-tb.y / alpha, tb.x / alpha), bm[c]);  // (i b / alpha) / beta-
  }
  // edge weights between window entries j and j + 1 (zero across the face ends)
  double2 sw[4];
  for (int j = 0; j < 4; ++j)
    sw[j] = (in[j] && in[j + 1]) ? mk(0.5 * ih2 * (kap[j].x + kap[j + 1].x), 0.5 * ih2 * (kap[j].y + kap[j + 1].y))
                                 : mk(0.0, 0.0);
  // M[x][y] = beta+_x delta_xy + beta-_x C[x][y] for window rows x = 1 .. 3, |x - y| <= 1
  auto Mv = [&](int cx, int cy) -> double2 {
    if (!in[cx] || !in[cy]) return mk(0.0, 0.0);
    double2 C;
    if (cy == cx - 1) C = sw[cx - 1];
    else if (cy == cx + 1) C = sw[cx];
    else C = mk(-(sw[cx - 1].x + sw[cx].x), -(sw[cx - 1].y + sw[cx].y));
    double2 v = cmul(bm[cx], C);
    if (cx == cy) v = cadd(v, bp[cx]);
    return v;
  };
  // R row e: M[e][y] / beta-_y;  Sigma row e: sum_y R[e][y] M[y][z] - beta-_e delta_ez
  double2 R[3];
  for (int d = 0; d < 3; ++d) R[d] = in[d + 1] ? cdiv(Mv(2, d + 1), bm[d + 1]) : mk(0.0, 0.0);
  for (int z = 0; z < 5; ++z) {
    double2 v = mk(0.0, 0.0);
    for (int d = 0; d < 3; ++d) {
      const int y = d + 1;
      if (z >= y - 1 && z <= y + 1) cfma(v, R[d], Mv(y, z));
    }
    if (z == 2) v = mk(v.x - bm[2].x, v.y - bm[2].y);
    B.sg[z] = in[z] ? v : mk(0.0, 0.0);
  }
  for (int d = 0; d < 3; ++d) B.r[d] = R[d];
  B.t[0] = sw[1];
  B.t[1] = sw[2];
  band[q] = B;
}

// diag[s][l]: diagonal of A_s including every face term
__global__ void k_local_diag(Geom g, const double* m, const FaceTab* ft, const IfCoef* coef, const IfBand* band,
                             double2* diag) {
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
      const int q = F.in_off[f] + (f < 2 ? ly : lx);
      rho = coef[q].rho;
      // second-order transmission: -(C u)_e / h^2 adds (s_{e-1,e} + s_{e,e+1}) / h^2 to the diagonal
      const IfBand& B = band[q];
      d.x += (B.t[0].x + B.t[1].x) * ih2;
      d.y += (B.t[0].y + B.t[1].y) * ih2;
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
// The second-order transmission adds -s_{e,e+1} / h^2 between consecutive edge nodes of an
// interface face (vertical neighbours on W/E faces, horizontal ones on S/N faces).
__global__ void k_band_assemble(Geom g, const double2* diag, const FaceTab* ft, const IfBand* band, double2* ab,
                                int nsub) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)g.nloc * g.ldab;
  if (t >= per * nsub) return;
  const int s = (int)(t / per);
  const size_t rem = t - (size_t)s * per;
  const int j = (int)(rem / g.ldab), r = (int)(rem % g.ldab);
  const int i = r - g.kv + j;  // row of A
  const double ih2 = 1.0 / (g.h * g.h);
  const double off = -ih2;
  double2 v = mk(0.0, 0.0);
  if (i >= 0 && i < g.nloc) {
    const int d = i - j;
    const int lo = min(i, j);
    const int ly = lo / g.snx, lx = lo - ly * g.snx;
    auto tangential = [&](int f, int e) {  // subtract s_{e,e+1} / h^2 if face f carries data
      const int io = ft[s].in_off[f];
      if (io < 0) return;
      const double2 w = band[io + e].t[1];
      v.x -= w.x * ih2;
      v.y -= w.y * ih2;
    };
    if (d == 0) {
      v = diag[(size_t)s * g.nloc + j];
    } else if ((d == 1 && (j % g.snx) != g.snx - 1) || (d == -1 && (j % g.snx) != 0)) {
      v = mk(off, 0.0);
      if (ly == 0) tangential(FACE_S, lx);
      if (ly == g.sny - 1) tangential(FACE_N, lx);
    } else if (d == g.snx || d == -g.snx) {
      v = mk(off, 0.0);
      if (lx == 0) tangential(FACE_W, ly);
      if (lx == g.snx - 1) tangential(FACE_E, ly);
    }
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

hipError_t launch_if_coef(const Geom& g, const double* m, const int32_t* pos_tab, double2 ta, IfCoef* coef,
                          hipStream_t st) {
  if (g.nif == 0) return hipSuccess;
  hipLaunchKernelGGL(k_if_coef, dim3((g.nif + 255) / 256), dim3(256), 0, st, g, m, pos_tab, ta, coef);
  return hipGetLastError();
}

hipError_t launch_if_band(const Geom& g, const double* m, const int32_t* pos_tab, int order, double2 ta, double2 tb,
                          const IfCoef* coef, IfBand* band, hipStream_t st) {
  if (g.nif == 0) return hipSuccess;
  hipLaunchKernelGGL(k_if_band, dim3((g.nif + 255) / 256), dim3(256), 0, st, g, m, pos_tab, order, ta, tb, coef, band);
  return hipGetLastError();
}

hipError_t launch_local_diag(const Geom& g, const double* m, const FaceTab* ft, const IfCoef* coef, const IfBand* band,
                             double2* diag, hipStream_t st) {
  const size_t n = (size_t)g.n1 * g.n2 * g.nloc;
  hipLaunchKernelGGL(k_local_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, m, ft, coef, band, diag);
  return hipGetLastError();
}

hipError_t launch_band_assemble(const Geom& g, const double2* diag, const FaceTab* ft, const IfBand* band, double2* ab,
                                int nsub, hipStream_t st) {
  const size_t n = (size_t)nsub * g.nloc * g.ldab;
  hipLaunchKernelGGL(k_band_assemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, diag, ft, band, ab, nsub);
  return hipGetLastError();
}
