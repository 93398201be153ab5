// Pade transmission condition (paper Sec. 7: the experiments prescribe a Pade-type high-order
// absorbing condition with N_pade = 8 auxiliary fields and branch rotation phi = pi/3 on every
// interface) in the dense operator form.
//
// On an interface face the impedance alpha of the first-order face template becomes the dense
// symmetric matrix X = K^1/2 R(D) K^1/2 along the face: R is the rotated Pade approximation of
// sqrt(1 + Z), C0 + sum_l A_l Z (1 + B_l Z)^-1 (Milinazzo, Zala and Brooke 1997), with the
// auxiliary fields eliminated, Z = D the tangential second difference d_tau(kappa^-2 d_tau) with
// Neumann face ends, K = diag(kappa) the interface wavenumbers.  With Q = (I/h - (i/2) X)^-1:
//   the face nodes' rows of A_s gain the dense block -rho / h^2, rho = (2/h) Q - I,
//   incoming data enter the right-hand side as J g, J = Q / h^2,
//   the data sent across are -rho g - sigma u_face, sigma = (4/h)(Q/h - I).
// The band factorisation keeps the Robin closure (A_b, first-order rho1 on the diagonal), and the
// dense blocks are a correction of rank at most L = 2 sub_nx + 2 sub_ny on the edge nodes:
//   A_s = A_b + U C U^T,  C = blockdiag_f(-(rho_f - rho1_f) / h^2),
// U the edge-node selector (one column per local interface position).  With Y = A_b^-1 U (the
// unit-datum solves that the dense form computes anyway, stored as W), M = U^T Y and
// G = I + C M, A_s^-1 U = Y G^-1 (Woodbury: (A_b + U C U^T) Y G^-1 = U (I + C M) G^-1 = U), so
//   T_s = -P - Sigma M G^-1 J           (P, Sigma, J block-diagonal by face)
//   lifting        U^T A_s^-1 f = G^-T Y^T f,  b = -Sigma (G^-T Y^T f)    (A_s = A_s^T)
//   reconstruction u = v + Y G^-1 (J g - C U^T v),  v = A_b^-1 f           (Woodbury again)
// so every operator of the method keeps its dense form, and the banded solves stay banded.
//
// Face blocks ("fb") are stored per subdomain as four dense blocks, faces W, E, S, N in the
// local interface order, block f row-major len_f x len_f at face_off2(f) (zero for outer faces).
#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "hbj_internal.h"

namespace {

typedef std::complex<double> zc;

// ---------------------------------------------------------------------------
// host: the face matrices of one face
// ---------------------------------------------------------------------------

void pade_coefficients(int npade, double phi, zc* c0, std::vector<zc>* A, std::vector<zc>* B) {
  const double pi = 3.14159265358979323846;
  const zc w0 = std::exp(zc(0.0, -phi)) - 1.0;  // the rotated variable at z = 0
  zc sum = 0.0;
  A->assign(npade, 0.0);
  B->assign(npade, 0.0);
  for (int l = 1; l <= npade; ++l) {
    const double s = std::sin(l * pi / (2 * npade + 1)), c = std::cos(l * pi / (2 * npade + 1));
    const double a = 2.0 / (2 * npade + 1) * s * s, b = c * c;
    const zc den = 1.0 + b * w0;
    sum += a * w0 / den;
    (*A)[l - 1] = std::exp(zc(0.0, -0.5 * phi)) * a / (den * den);
    (*B)[l - 1] = std::exp(zc(0.0, -phi)) * b / den;
  }
  *c0 = std::exp(zc(0.0, 0.5 * phi)) * (1.0 + sum);
}

// In-place inverse of the n x n row-major matrix a by Gauss-Jordan elimination with partial
// pivoting; false if a pivot is exactly zero.
bool invert_host(std::vector<zc>& a, int n) {
  std::vector<int> perm(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = -1.0;
    for (int i = k; i < n; ++i) {
      const double v = std::abs(a[(size_t)i * n + k].real()) + std::abs(a[(size_t)i * n + k].imag());
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0) return false;
    perm[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
    const zc inv = 1.0 / a[(size_t)k * n + k];
    a[(size_t)k * n + k] = 1.0;
    for (int j = 0; j < n; ++j) a[(size_t)k * n + j] *= inv;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const zc f = a[(size_t)i * n + k];
      if (f == 0.0) continue;
      a[(size_t)i * n + k] = 0.0;
      for (int j = 0; j < n; ++j) a[(size_t)i * n + j] -= f * a[(size_t)k * n + j];
    }
  }
  for (int k = n - 1; k >= 0; --k)
    if (perm[k] != k)
      for (int i = 0; i < n; ++i) std::swap(a[(size_t)i * n + k], a[(size_t)i * n + perm[k]]);
  return true;
}

// Face matrices of a face with wavenumbers kappa[0..n) and Robin diagonal rho1 of the band
// factors: rho, sigma, inj (= J) and the correction corr = -(rho - diag(rho1)) / h^2, each
// row-major n x n, written at the four outputs.
bool face_blocks(const double* kappa, const double2* rho1, int n, double h, int npade, double phi, double2* rho,
                 double2* sigma, double2* inj, double2* corr) {
  zc c0;
  std::vector<zc> A, B;
  pade_coefficients(npade, phi, &c0, &A, &B);
  // tridiagonal D: off-diagonal w_e between e and e+1, diagonal -(w_{e-1} + w_e)
  std::vector<double> w(std::max(n - 1, 0));
  for (int e = 0; e + 1 < n; ++e) w[e] = 1.0 / (h * h * kappa[e] * kappa[e + 1]);
  std::vector<double> dd(n, 0.0);
  for (int e = 0; e + 1 < n; ++e) {
    dd[e] -= w[e];
    dd[e + 1] -= w[e];
  }
  // R = C0 I + sum_l (A_l / B_l) (I - (I + B_l D)^-1): columns by a complex tridiagonal solve
  std::vector<zc> R((size_t)n * n, 0.0);
  for (int e = 0; e < n; ++e) R[(size_t)e * n + e] = c0;
  std::vector<zc> cp(n), z(n);
  for (size_t l = 0; l < A.size(); ++l) {
    const zc bl = B[l], al = A[l];
    for (int j = 0; j < n; ++j) {
      // (I + bl D) z = e_j by the Thomas algorithm: sub/super diagonal bl w, diagonal 1 + bl dd
      for (int e = 0; e < n; ++e) {
        const zc diag = 1.0 + bl * dd[e];
        const zc lo = e > 0 ? bl * w[e - 1] : 0.0;
        const zc up = e + 1 < n ? bl * w[e] : 0.0;
        const zc rhs = (e == j) ? 1.0 : 0.0;
        const zc den = e > 0 ? diag - lo * cp[e - 1] : diag;
        cp[e] = up / den;
        z[e] = (e > 0 ? rhs - lo * z[e - 1] : rhs) / den;
      }
      for (int e = n - 2; e >= 0; --e) z[e] -= cp[e] * z[e + 1];
      for (int e = 0; e < n; ++e) R[(size_t)e * n + j] += (al / bl) * ((e == j ? 1.0 : 0.0) - z[e]);
    }
  }
  // beta- = I/h - (i/2) K^1/2 R K^1/2, Q = beta-^-1
  std::vector<zc> Q((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const zc x = std::sqrt(kappa[i]) * R[(size_t)i * n + j] * std::sqrt(kappa[j]);
      Q[(size_t)i * n + j] = (i == j ? zc(1.0 / h, 0.0) : zc(0.0, 0.0)) - zc(0.0, 0.5) * x;
    }
  if (!invert_host(Q, n)) return false;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t o = (size_t)i * n + j;
      const zc q = Q[o];
      const zc id = (i == j) ? 1.0 : 0.0;
      const zc r = (2.0 / h) * q - id;
      const zc s = (4.0 / h) * (q / h - id);
      const zc jn = q / (h * h);
      const zc r1 = (i == j) ? zc(rho1[i].x, rho1[i].y) : zc(0.0, 0.0);
      const zc cr = -(r - r1) / (h * h);
      rho[o] = mk(r.real(), r.imag());
      sigma[o] = mk(s.real(), s.imag());
      inj[o] = mk(jn.real(), jn.imag());
      corr[o] = mk(cr.real(), cr.imag());
    }
  return true;
}

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------

// offset of face f's block within a subdomain's face blocks
__host__ __device__ inline size_t face_off2(const Geom& g, int f) {
  const size_t a = (size_t)g.sny * g.sny, b = (size_t)g.snx * g.snx;
  return f == 0 ? 0 : f == 1 ? a : f == 2 ? 2 * a : 2 * a + b;
}

constexpr int kPT = 256;  // threads of the row kernels

// out[s][r][c] = addI delta_rc + sum_e' FB_s,f(r)[e(r)][e'] X[s][xrow(f, e')][c]: a face-block
// matrix times a dense one.  X rows are taken at the edge nodes (NODES: X = W [nloc][L]) or at the
// local interface positions (X is L x L).  Rows of faces without a neighbour hold addI delta_rc.
template <bool NODES>
__global__ __launch_bounds__(kPT) void k_fb_left(Geom g, const FaceTab* ft, const double2* __restrict__ fb,
                                                 const double2* __restrict__ X, int addI, double2* out) {
  const int r = blockIdx.x, s = blockIdx.y;
  const int L = local_if_len(g);
  int f, e;
  local_if_face(g, r, &f, &e);
  const int len = face_len(g, f);
  const bool has = pick4(ft[s].in_off, f) >= 0;
  const double2* fr = fb + (size_t)s * (2 * (size_t)g.sny * g.sny + 2 * (size_t)g.snx * g.snx) + face_off2(g, f) +
                      (size_t)e * len;
  const size_t xs = NODES ? (size_t)g.nloc * L : (size_t)L * L;
  const double2* Xs = X + (size_t)s * xs;
  __shared__ double2 frow[256];
  for (int q = threadIdx.x; q < len; q += kPT) frow[q] = has ? fr[q] : mk(0.0, 0.0);
  __syncthreads();
  for (int c = threadIdx.x; c < L; c += kPT) {
    double2 acc = mk((addI && c == r) ? 1.0 : 0.0, 0.0);
    if (has) {
      for (int q = 0; q < len; ++q) {
        const int xr = NODES ? face_node(g, f, q) : face_off(g, f) + q;
        cfma(acc, frow[q], Xs[(size_t)xr * L + c]);
      }
    }
    out[((size_t)s * L + r) * L + c] = acc;
  }
}

// out[s][r][c] = sum_e' X[s][r][off(f(c)) + e'] FB_s,f(c)[e'][e(c)]: a dense matrix times a
// face-block one (columns of faces without a neighbour are zero)
__global__ __launch_bounds__(kPT) void k_fb_right(Geom g, const FaceTab* ft, const double2* __restrict__ X,
                                                  const double2* __restrict__ fb, double2* out) {
  const int r = blockIdx.x, s = blockIdx.y;
  const int L = local_if_len(g);
  __shared__ double2 xrow[1024];
  const double2* xr = X + ((size_t)s * L + r) * L;
  for (int c = threadIdx.x; c < L; c += kPT) xrow[c] = xr[c];
  __syncthreads();
  const double2* fs = fb + (size_t)s * (2 * (size_t)g.sny * g.sny + 2 * (size_t)g.snx * g.snx);
  for (int c = threadIdx.x; c < L; c += kPT) {
    int f, e;
    local_if_face(g, c, &f, &e);
    const int len = face_len(g, f), off = face_off(g, f);
    double2 acc = mk(0.0, 0.0);
    if (pick4(ft[s].in_off, f) >= 0) {
      const double2* fc = fs + face_off2(g, f) + e;
      for (int q = 0; q < len; ++q) cfma(acc, xrow[off + q], fc[(size_t)q * len]);
    }
    out[((size_t)s * L + r) * L + c] = acc;
  }
}

// out[s] = A[s] B[s] with A's row r taken from W[s][node(r)] (the edge values M = U^T Y) and B
// L x L; 64 x 64 output tiles, 16-deep k-slices staged in LDS, 4 x 4 outputs per thread.
constexpr int GT = 64, GK = 16;
__global__ __launch_bounds__(256) void k_gemm_edge_rows(Geom g, const double2* __restrict__ W,
                                                        const double2* __restrict__ B, double2* out) {
  const int L = local_if_len(g);
  const int s = blockIdx.z, r0 = blockIdx.y * GT, c0 = blockIdx.x * GT;
  const double2* Ws = W + (size_t)s * g.nloc * L;
  const double2* Bs = B + (size_t)s * L * L;
  __shared__ double2 As[GT][GK + 1];
  __shared__ double2 Bsh[GK][GT + 1];
  __shared__ int arow[GT];
  if (threadIdx.x < GT) {
    const int r = r0 + threadIdx.x;
    int f = 0, e = 0;
    if (r < L) local_if_face(g, r, &f, &e);
    arow[threadIdx.x] = r < L ? face_node(g, f, e) : -1;
  }
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;  // rows tr + 16 i, columns tc + 16 j
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk(0.0, 0.0);
  __syncthreads();
  for (int k0 = 0; k0 < L; k0 += GK) {
    for (int t = threadIdx.x; t < GT * GK; t += 256) {
      const int i = t / GK, kk = t % GK;
      const int row = arow[i], k = k0 + kk;
      As[i][kk] = (row >= 0 && k < L) ? Ws[(size_t)row * L + k] : mk(0.0, 0.0);
    }
    for (int t = threadIdx.x; t < GK * GT; t += 256) {
      const int kk = t / GT, j = t % GT;
      const int k = k0 + kk, c = c0 + j;
      Bsh[kk][j] = (k < L && c < L) ? Bs[(size_t)k * L + c] : mk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GK; ++kk) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[tr + 16 * i][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bsh[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + tr + 16 * i, c = c0 + tc + 16 * j;
      if (r < L && c < L) out[((size_t)s * L + r) * L + c] = acc[i][j];
    }
}

// In-place inverse of every A[s] (L x L, row-major) by Gauss-Jordan elimination with partial
// pivoting (pivot: first maximum of |re| + |im|), one workgroup per matrix; info[s] = k + 1 if the
// k-th pivot is exactly zero (the matrix is singular; the output is then invalid).  piv[s][k] is
// the row exchanged with row k, undone on the columns at the end.
constexpr int GJT = 1024;
__global__ __launch_bounds__(GJT) void k_gj_inverse(int L, double2* A, int32_t* piv, int32_t* info) {
  const int s = blockIdx.x;
  double2* a = A + (size_t)s * L * L;
  int32_t* pv = piv + (size_t)s * L;
  __shared__ double2 colk[1024], rowk[1024];
  __shared__ double rv[GJT / 64];
  __shared__ int ri[GJT / 64];
  __shared__ int s_p;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int bad = 0;
  for (int k = 0; k < L; ++k) {
    // 1. pivot: first row of maximal |re| + |im| among rows k..L-1 of column k
    double best = -1.0;
    int bi = L;
    for (int i = k + (int)threadIdx.x; i < L; i += GJT) {
      const double v = cabs1(a[(size_t)i * L + k]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { rv[wv] = best; ri[wv] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = rv[0];
      int p = ri[0];
      for (int w = 1; w < GJT / 64; ++w)
        if (rv[w] > b || (rv[w] == b && ri[w] < p)) { b = rv[w]; p = ri[w]; }
      if (!(b > 0.0)) p = k;  // exactly singular: keep going on row k, the result is flagged
      s_p = p;
      pv[k] = p;
    }
    __syncthreads();
    const int p = s_p;
    // 2. exchange rows k and p; take the pivot row and column k (old values) into LDS
    for (int j = threadIdx.x; j < L; j += GJT) {
      const double2 vk = a[(size_t)k * L + j], vp = a[(size_t)p * L + j];
      if (p != k) a[(size_t)p * L + j] = vk;
      rowk[j] = vp;  // the new row k
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += GJT) colk[i] = (i == k) ? rowk[k] : (i == p ? a[(size_t)i * L + k] : a[(size_t)i * L + k]);
    __syncthreads();
    // 3. scale the pivot row: row k becomes (row k with a_kk := 1) / pivot
    const double2 pivot = rowk[k];
    if (cabs1(pivot) == 0.0) bad = bad ? bad : k + 1;
    const double2 pinv = (cabs1(pivot) == 0.0) ? mk(0.0, 0.0) : cdiv(mk(1.0, 0.0), pivot);
    __syncthreads();
    for (int j = threadIdx.x; j < L; j += GJT) {
      const double2 v = (j == k) ? mk(1.0, 0.0) : rowk[j];
      const double2 sv = cmul(v, pinv);
      rowk[j] = sv;
      a[(size_t)k * L + j] = sv;
    }
    __syncthreads();
    // 4. eliminate column k from every other row: a_ij := (j == k ? 0 : a_ij) - a_ik rowk_j
    for (int t = threadIdx.x; t < L * L; t += GJT) {
      const int i = t / L, j = t - i * L;
      if (i == k) continue;
      const double2 f = colk[i];
      double2 v = (j == k) ? mk(0.0, 0.0) : a[t];
      v.x -= f.x * rowk[j].x - f.y * rowk[j].y;
      v.y -= f.x * rowk[j].y + f.y * rowk[j].x;
      a[t] = v;
    }
    __syncthreads();
  }
  // 5. undo the row exchanges on the columns, last first
  for (int k = L - 1; k >= 0; --k) {
    const int p = pv[k];
    if (p != k)
      for (int i = threadIdx.x; i < L; i += GJT) {
        const double2 t = a[(size_t)i * L + k];
        a[(size_t)i * L + k] = a[(size_t)i * L + p];
        a[(size_t)i * L + p] = t;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) info[s] = bad;
}

// T_s[t_index(r, c)] = -P_f(r)[e(r)][e(c)] [f(c) = f(r)] - sum_e' Sigma_f(r)[e(r)][e'] X[s][off(f(r)) + e'][c]
// for rows of faces with a neighbour (other rows: 0); X = M G^-1 J.
__global__ __launch_bounds__(kPT) void k_pade_T(Geom g, const FaceTab* ft, const double2* __restrict__ fbP,
                                                const double2* __restrict__ fbS, const double2* __restrict__ X,
                                                double2* T) {
  const int r = blockIdx.x, s = blockIdx.y;
  const int L = local_if_len(g);
  int f, e;
  local_if_face(g, r, &f, &e);
  const int len = face_len(g, f), off = face_off(g, f);
  const bool has = pick4(ft[s].in_off, f) >= 0;
  const size_t fbs = 2 * (size_t)g.sny * g.sny + 2 * (size_t)g.snx * g.snx;
  const double2* sr = fbS + (size_t)s * fbs + face_off2(g, f) + (size_t)e * len;
  const double2* pr = fbP + (size_t)s * fbs + face_off2(g, f) + (size_t)e * len;
  __shared__ double2 srow[256];
  for (int q = threadIdx.x; q < len; q += kPT) srow[q] = has ? sr[q] : mk(0.0, 0.0);
  __syncthreads();
  const double2* Xs = X + (size_t)s * L * L;
  double2* Ts = T + (size_t)s * t_per_sub(g);
  for (int c = threadIdx.x; c < L; c += kPT) {
    double2 acc = mk(0.0, 0.0);
    if (has) {
      for (int q = 0; q < len; ++q) cfma(acc, srow[q], Xs[(size_t)(off + q) * L + c]);
      if (c >= off && c < off + len) acc = cadd(acc, pr[c - off]);
    }
    Ts[t_index(L, r, c)] = mk(-acc.x, -acc.y);
  }
}

// Lifting of the Pade form, one workgroup per subdomain and group of up to PRB right-hand sides (G^-1
// is read once per group): y = the sum of the chunk partials of W^T f (chunk order), y' = G^-T y,
// b at the outgoing positions of every face with a neighbour = -Sigma_f y'_f (0 for right-hand sides
// without a source in the subdomain).
constexpr int PRB = 4;
__global__ __launch_bounds__(1024) void k_pade_lift(Geom g, const FaceTab* ft, const double2* __restrict__ fbS,
                                                    const double2* __restrict__ Ginv, const int32_t* nz,
                                                    const double2* part, int nchunk, int nrhs, double2* b) {
  const int s = blockIdx.x, r0 = blockIdx.y * PRB;
  const int ndom = g.n1 * g.n2;
  const int L = local_if_len(g);
  const int nr = min(PRB, nrhs - r0);
  const FaceTab F = ft[s];
  __shared__ double2 y[PRB][1024], yp[PRB][1024];
  bool any = false;
  for (int k = 0; k < nr; ++k) any |= nz[(size_t)(r0 + k) * ndom + s] != 0;
  for (int k = 0; k < nr; ++k) {
    const bool has = nz[(size_t)(r0 + k) * ndom + s] != 0;
    for (int q = threadIdx.x; q < L; q += blockDim.x) {
      double2 acc = mk(0.0, 0.0);
      if (has) {
        const double2* ps = part + (size_t)((r0 + k) * ndom + s) * nchunk * L + q;
        for (int c = 0; c < nchunk; ++c) acc = cadd(acc, ps[(size_t)c * L]);
      }
      y[k][q] = acc;
    }
  }
  __syncthreads();
  const double2* Gs = Ginv + (size_t)s * L * L;
  constexpr int QU = 8;  // rows of G^-1 whose loads are in flight together
  for (int c = threadIdx.x; c < L; c += blockDim.x) {
    double2 acc[PRB];
#pragma unroll
    for (int k = 0; k < PRB; ++k) acc[k] = mk(0.0, 0.0);
    if (any)
      for (int q0 = 0; q0 < L; q0 += QU) {
        double2 gv[QU];
#pragma unroll
        for (int u = 0; u < QU; ++u) gv[u] = Gs[(size_t)min(q0 + u, L - 1) * L + c];
#pragma unroll
        for (int u = 0; u < QU; ++u)
          if (q0 + u < L)
#pragma unroll
            for (int k = 0; k < PRB; ++k)
              if (k < nr) cfma(acc[k], gv[u], y[k][q0 + u]);
      }
#pragma unroll
    for (int k = 0; k < PRB; ++k) yp[k][c] = acc[k];
  }
  __syncthreads();
  const size_t fbs = 2 * (size_t)g.sny * g.sny + 2 * (size_t)g.snx * g.snx;
  for (int row = threadIdx.x; row < L; row += blockDim.x) {
    int f, e;
    local_if_face(g, row, &f, &e);
    const int oo = pick4(F.out_off, f);
    if (oo < 0) continue;
    const int len = face_len(g, f), off = face_off(g, f);
    const double2* sr = fbS + (size_t)s * fbs + face_off2(g, f) + (size_t)e * len;
    double2 acc[PRB];
#pragma unroll
    for (int k = 0; k < PRB; ++k) acc[k] = mk(0.0, 0.0);
    for (int q = 0; q < len; ++q) {
      const double2 sv = sr[q];
#pragma unroll
      for (int k = 0; k < PRB; ++k)
        if (k < nr) cfma(acc[k], sv, yp[k][off + q]);
    }
    for (int k = 0; k < nr; ++k) b[(size_t)(r0 + k) * g.nif + oo + e] = mk(-acc[k].x, -acc[k].y);
  }
}

// Reconstruction data of the Pade form, in two passes.  Pass 1, one workgroup per (subdomain,
// right-hand side): q = J g - C U^T v on the faces with a neighbour (v = the source part already in
// u, for subdomains with a source; 0 on outer faces), a wavefront per entry of q reading its rows of
// J and C along the face.  Pass 2, one workgroup per (subdomain, group of up to PRB right-hand
// sides, chunk of kRecRows rows of G^-1): t = G^-1 q for the chunk's rows, a wavefront per row of
// G^-1 (read once per group), and gt = t / inj at the subdomain's incoming positions, so that the
// reconstruction products u += W (inj gt) add Y G^-1 q.
__global__ __launch_bounds__(512) void k_pade_recon_q(Geom g, const FaceTab* ft, const double2* __restrict__ fbJ,
                                                      const double2* __restrict__ fbC, const double2* gin,
                                                      const int32_t* nz, const double2* u, double2* qbuf) {
  const int s = blockIdx.x, r = blockIdx.y;
  const int ndom = g.n1 * g.n2;
  const int L = local_if_len(g);
  const bool has = nz[(size_t)r * ndom + s] != 0;
  const FaceTab F = ft[s];
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
  __shared__ double2 gl[1024], vl[1024];
  for (int c = threadIdx.x; c < L; c += blockDim.x) {
    int f, e;
    local_if_face(g, c, &f, &e);
    const int io = pick4(F.in_off, f);
    gl[c] = io >= 0 ? gin[(size_t)r * g.nif + io + e] : mk(0.0, 0.0);
    double2 v = mk(0.0, 0.0);
    if (has && io >= 0) {
      const int p = face_node(g, f, e);
      const int ly = p / g.snx, lx = p - ly * g.snx;
      v = u[(size_t)r * g.nx * g.ny + (size_t)(y0 + ly) * g.nx + x0 + lx];
    }
    vl[c] = v;
  }
  __syncthreads();
  const size_t fbs = 2 * (size_t)g.sny * g.sny + 2 * (size_t)g.snx * g.snx;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double2* qs = qbuf + ((size_t)r * ndom + s) * L;
  for (int c = wv; c < L; c += nw) {
    int f, e;
    local_if_face(g, c, &f, &e);
    double2 acc = mk(0.0, 0.0);
    if (pick4(F.in_off, f) >= 0) {
      const int len = face_len(g, f), off = face_off(g, f);
      const double2* jr = fbJ + (size_t)s * fbs + face_off2(g, f) + (size_t)e * len;
      const double2* cr = fbC + (size_t)s * fbs + face_off2(g, f) + (size_t)e * len;
      for (int m = lane; m < len; m += 64) {
        cfma(acc, jr[m], gl[off + m]);
        const double2 cv = cr[m];
        cfma(acc, mk(-cv.x, -cv.y), vl[off + m]);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        acc.x += __shfl_xor(acc.x, o);
        acc.y += __shfl_xor(acc.y, o);
      }
    }
    if (lane == 0) qs[c] = acc;
  }
}

constexpr int kRecRows = 64;
__global__ __launch_bounds__(512) void k_pade_recon_t(Geom g, const FaceTab* ft, const IfCoef* coef,
                                                      const double2* __restrict__ Ginv, const double2* qbuf, int nrhs,
                                                      double2* gt) {
  const int s = blockIdx.x, r0 = blockIdx.y * PRB, row0 = blockIdx.z * kRecRows;
  const int ndom = g.n1 * g.n2;
  const int L = local_if_len(g);
  const int nr = min(PRB, nrhs - r0);
  const FaceTab F = ft[s];
  __shared__ double2 q[PRB][1024];
  for (int k = 0; k < nr; ++k)
    for (int c = threadIdx.x; c < L; c += blockDim.x) q[k][c] = qbuf[((size_t)(r0 + k) * ndom + s) * L + c];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const double2* Gs = Ginv + (size_t)s * L * L;
  const int row1 = min(L, row0 + kRecRows);
  for (int row = row0 + wv; row < row1; row += nw) {
    double2 acc[PRB];
#pragma unroll
    for (int k = 0; k < PRB; ++k) acc[k] = mk(0.0, 0.0);
    for (int c = lane; c < L; c += 64) {
      const double2 gv = Gs[(size_t)row * L + c];
#pragma unroll
      for (int k = 0; k < PRB; ++k)
        if (k < nr) cfma(acc[k], gv, q[k][c]);
    }
#pragma unroll
    for (int k = 0; k < PRB; ++k)
      if (k < nr)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          acc[k].x += __shfl_xor(acc[k].x, off);
          acc[k].y += __shfl_xor(acc[k].y, off);
        }
    if (lane == 0) {
      int f, e;
      local_if_face(g, row, &f, &e);
      const int io = pick4(F.in_off, f);
      if (io >= 0)
        for (int k = 0; k < nr; ++k) gt[(size_t)(r0 + k) * g.nif + io + e] = cdiv(acc[k], coef[io + e].inj);
    }
  }
}

}  // namespace

size_t pade_fb_per_sub(const Geom& g) { return 2 * (size_t)g.sny * g.sny + 2 * (size_t)g.snx * g.snx; }

int pade_face_blocks(const Geom& g, const FaceTab* ft_host, const double* m_host, const IfCoef* coef_host,
                     int npade, double phi, double2* rho, double2* sigma, double2* inj, double2* corr) {
  const int ndom = g.n1 * g.n2;
  const size_t fbs = pade_fb_per_sub(g);
  std::fill(rho, rho + fbs * ndom, mk(0.0, 0.0));
  std::fill(sigma, sigma + fbs * ndom, mk(0.0, 0.0));
  std::fill(inj, inj + fbs * ndom, mk(0.0, 0.0));
  std::fill(corr, corr + fbs * ndom, mk(0.0, 0.0));
  // work items: every (subdomain, face) with a neighbour
  std::vector<std::pair<int, int>> items;
  for (int s = 0; s < ndom; ++s)
    for (int f = 0; f < 4; ++f)
      if (ft_host[s].in_off[f] >= 0) items.emplace_back(s, f);
  std::vector<int> ok(items.size(), 1);
  auto work = [&](size_t i0, size_t stride) {
    std::vector<double> kappa;
    std::vector<double2> rho1;
    for (size_t i = i0; i < items.size(); i += stride) {
      const int s = items[i].first, f = items[i].second;
      const int len = face_len(g, f);
      const int i1 = s % g.n1, i2 = s / g.n1;
      kappa.assign(len, 0.0);
      rho1.assign(len, mk(0.0, 0.0));
      for (int e = 0; e < len; ++e) {
        // the two nodes of the face at entry e: p inside s, q across the face
        int px, py, qx, qy;
        if (f < 2) {
          py = qy = i2 * g.sny + e;
          px = f == 0 ? i1 * g.snx : i1 * g.snx + g.snx - 1;
          qx = f == 0 ? px - 1 : px + 1;
        } else {
          px = qx = i1 * g.snx + e;
          py = f == 2 ? i2 * g.sny : i2 * g.sny + g.sny - 1;
          qy = f == 2 ? py - 1 : py + 1;
        }
        const double mp = m_host[(size_t)py * g.nx + px], mq = m_host[(size_t)qy * g.nx + qx];
        kappa[e] = g.k * std::sqrt(0.5 * (mp + mq));
        rho1[e] = coef_host[ft_host[s].in_off[f] + e].rho;
      }
      const size_t o = (size_t)s * fbs + face_off2(g, f);
      if (!face_blocks(kappa.data(), rho1.data(), len, g.h, npade, phi, rho + o, sigma + o, inj + o, corr + o))
        ok[i] = 0;
    }
  };
  const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nth; ++t) th.emplace_back(work, (size_t)t, (size_t)nth);
  work(0, nth);
  for (auto& t : th) t.join();
  return std::all_of(ok.begin(), ok.end(), [](int v) { return v != 0; }) ? 0 : -1;
}

hipError_t launch_pade_T(const Geom& g, const FaceTab* ft, const double2* W, const double2* fbP, const double2* fbS,
                         const double2* fbJ, const double2* fbC, double2* Ginv, double2* work, int32_t* piv,
                         int32_t* info, double2* T, hipStream_t st) {
  const int L = local_if_len(g), ndom = g.n1 * g.n2;
  if (L > 1024 || face_len(g, 0) > 256 || face_len(g, 2) > 256) return hipErrorInvalidValue;
  // G = I + C M (M = edge rows of W), inverted in place
  hipLaunchKernelGGL((k_fb_left<true>), dim3(L, ndom), dim3(kPT), 0, st, g, ft, fbC, W, 1, Ginv);
  hipLaunchKernelGGL(k_gj_inverse, dim3(ndom), dim3(GJT), 0, st, L, Ginv, piv, info);
  // Z = G^-1 J into work, then X = M Z into the upper half of work, then T
  double2* Z = work;
  double2* X = work + (size_t)ndom * L * L;
  hipLaunchKernelGGL(k_fb_right, dim3(L, ndom), dim3(kPT), 0, st, g, ft, Ginv, fbJ, Z);
  hipLaunchKernelGGL(k_gemm_edge_rows, dim3((L + GT - 1) / GT, (L + GT - 1) / GT, ndom), dim3(256), 0, st, g, W, Z, X);
  hipLaunchKernelGGL(k_pade_T, dim3(L, ndom), dim3(kPT), 0, st, g, ft, fbP, fbS, X, T);
  return hipGetLastError();
}

hipError_t launch_pade_lift(const Geom& g, const FaceTab* ft, const double2* fbS, const double2* Ginv,
                            const int32_t* nz, const double2* part, int nchunk, int nrhs, double2* b, hipStream_t st) {
  const int L = local_if_len(g);
  if (L > 1024) return hipErrorInvalidValue;
  const int nt = std::min(1024, (L + 63) / 64 * 64);
  hipLaunchKernelGGL(k_pade_lift, dim3(g.n1 * g.n2, (nrhs + PRB - 1) / PRB), dim3(nt), 0, st, g, ft, fbS, Ginv, nz, part,
                     nchunk, nrhs, b);
  return hipGetLastError();
}

hipError_t launch_pade_recon_prep(const Geom& g, const FaceTab* ft, const IfCoef* coef, const double2* fbJ,
                                  const double2* fbC, const double2* Ginv, const double2* gin, const int32_t* nz,
                                  const double2* u, int nrhs, double2* qbuf, double2* gt, hipStream_t st) {
  const int L = local_if_len(g);
  if (L > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pade_recon_q, dim3(g.n1 * g.n2, nrhs), dim3(512), 0, st, g, ft, fbJ, fbC, gin, nz, u, qbuf);
  const dim3 grid(g.n1 * g.n2, (nrhs + PRB - 1) / PRB, (L + kRecRows - 1) / kRecRows);
  hipLaunchKernelGGL(k_pade_recon_t, grid, dim3(512), 0, st, g, ft, coef, Ginv, qbuf, nrhs, gt);
  return hipGetLastError();
}
