// Block Gram-Schmidt of the s-step Arnoldi cycle of (F)GMRES on the interface system (complex128).
//
// A cycle of s steps first builds the Krylov vectors y_{i+1} = (I - S) P^{-1} y_i - y_i from
// y_0 = v_k (a Newton basis with the single shift 1: the preconditioned operator is close to the
// identity, and the vectors of this basis stay far from parallel), each with one preconditioner and
// one operator launch as in a single step.  The s new vectors Y = [y_1 .. y_s] are then made
// orthonormal against V_0..V_k and among themselves in one inner-product pass and one update pass
// over the basis: C = V^H Y and the Gram matrix Y^H Y in the first, P = Y^H Y - C^H C = R^H R
// (Cholesky, after a diagonal scaling) in between, and Q = (Y - V C) R^{-1} in place of Y in the
// second (block classical Gram-Schmidt with the Pythagorean form of the Cholesky QR: Hoemmen,
// Communication-avoiding Krylov subspace methods, PhD thesis, UC Berkeley 2010; Carson, Lund,
// Rozloznik and Thomas, Block Gram-Schmidt algorithms and their stability properties, Linear
// Algebra Appl. 638, 2022).  The Hessenberg columns of the s steps follow on the host from C, R
// and the recurrence; in exact arithmetic the iterates are those of s single Arnoldi steps.
//
// Vectors come in column blocks [ncol][n] (one column per right-hand side); V_i starts at
// V + i vstride.  Every reduction has a fixed order (deterministic results).
#include "hbj_internal.h"

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
constexpr int kSB = kSstepMax;  // block steps at most (columns of Y)
constexpr int BW = 4;           // wavefronts per workgroup of the inner-product pass
constexpr int kTiles = kSstepMaxBasis / 16;

// Inner products D[i][l] = V_i^H Y_l (V_{k1 + l} = Y_l) for i < nvt = k1 + sb and l < kSB, per
// column, as partial sums over the positions of one workgroup:
// part[((col * nchunk + chunk) * nvt + i) * kSB + l].
// f64 MFMA 16x16x4 with the positions as the contraction index: A = the real or the imaginary
// parts of 16 basis vectors (lane (i, kk) holds vector 16 t + i), B = the real parts of Y_0..Y_7
// in its columns 0-7 and the imaginary parts in columns 8-15 (lane (c, kk)); then
// Re D = (Re V)^T (Re Y) + (Im V)^T (Im Y) and Im D = (Re V)^T (Im Y) - (Im V)^T (Re Y).
// Wavefront wv of workgroup chunk takes positions [(chunk BW + wv) pw, + pw) (pw a multiple of
// 16); k-step q of a batch of 16 positions p puts lane kk on position p + 4 q + kk in both
// operands.  Positions past the wavefront's range or the column's end, and columns l >= sb, get
// B = 0 (their loads clamped in bounds); basis vectors past nvt load the last one (rows never
// stored).  The wavefronts' tiles meet in LDS in a fixed order.
template <int NT>
__global__ __launch_bounds__(64 * BW) void k_bgs_dots(const double2* __restrict__ V, size_t vstride, int nvt,
                                                      int k1, int sb, int n, int pw, double2* __restrict__ part) {
  const int chunk = blockIdx.x, col = blockIdx.y, nchunk = gridDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, kk = lane >> 4;
  const long p0l = ((long)chunk * BW + wv) * pw;
  const int p0 = (int)min(p0l, (long)n), p1 = (int)min(p0l + pw, (long)n);
  const int l = r16 & 7;
  const bool take_re = r16 < 8, lok = l < sb;
  const double2* yb = V + (size_t)(k1 + (lok ? l : sb - 1)) * vstride + (size_t)col * n;
  const double2* va[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) va[t] = V + (size_t)min(16 * t + r16, nvt - 1) * vstride + (size_t)col * n;
  d4v a1[NT], a2[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    a1[t] = d4v{0.0, 0.0, 0.0, 0.0};
    a2[t] = d4v{0.0, 0.0, 0.0, 0.0};
  }
  for (int p = p0; p < p1; p += 16) {
    int pq[4];
    double2 bv[4], av[NT][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pq[q] = min(p + 4 * q + kk, n - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) bv[q] = yb[pq[q]];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) av[t][q] = va[t][pq[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool in = lok && (p + 4 * q + kk < p1);
      const double b = in ? (take_re ? bv[q].x : bv[q].y) : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        a1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t][q].x, b, a1[t], 0, 0, 0);
        a2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t][q].y, b, a2[t], 0, 0, 0);
      }
    }
  }
  // accumulator register r of lane (c, kk) holds row kk + 4 r, column c of the 16 x 16 tile
  __shared__ double red[BW][NT][2][256];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = (kk + 4 * r) * 16 + r16;
      red[wv][t][0][e] = a1[t][r];
      red[wv][t][1][e] = a2[t][r];
    }
  __syncthreads();
  double2* out = part + ((size_t)col * nchunk + chunk) * nvt * kSB;
  for (int o = threadIdx.x; o < nvt * kSB; o += 64 * BW) {
    const int i = o / kSB, c = o % kSB, t = i >> 4, row = i & 15;
    double rr = 0.0, ri = 0.0, ir = 0.0, ii = 0.0;  // (Re V . Re Y), (Re V . Im Y), (Im V . Re Y), (Im V . Im Y)
#pragma unroll
    for (int w = 0; w < BW; ++w) {
      rr += red[w][t][0][row * 16 + c];
      ri += red[w][t][0][row * 16 + c + 8];
      ir += red[w][t][1][row * 16 + c];
      ii += red[w][t][1][row * 16 + c + 8];
    }
    out[o] = mk(rr + ii, ri - ir);
  }
}

// Per column: D = the sum of the partials in chunk order, C = D[0..k1), the Gram matrix
// G[p][l] = D[k1 + p][l] = Y_p^H Y_l, P = G - C^H C, and the Cholesky factor R (upper, P = R^H R)
// computed on P scaled by 1/sqrt(G_pp G_ll) and scaled back; R^{-1} alongside.  Record of column
// col at coef + col ldc: R[p][l] at p kSB + l, R^{-1} at 64 + p kSB + l, at 128 the index b of the
// first pivot that failed (sb if none) as a double, and C[i][l] at 129 + i kSB + l.  A pivot fails
// when y_{b+1} has (relative to its norm) no component beyond 1e-13 outside the span of the basis
// and the earlier new vectors, or is zero: R's rows from b on are then zero, and so are the
// columns of R^{-1} from b on, which makes those vectors of Q zero.
constexpr int kRed = 256;
__global__ __launch_bounds__(kRed) void k_bgs_reduce(const double2* __restrict__ part, int nchunk, int nvt, int k1,
                                                     int sb, double2* __restrict__ coef, int ldc) {
  const int col = blockIdx.x;
  __shared__ double2 D[kSstepMaxBasis * kSB];
  __shared__ double2 P[kSB * kSB];
  const double2* pc = part + (size_t)col * nchunk * nvt * kSB;
  for (int o = threadIdx.x; o < nvt * kSB; o += kRed) {
    double2 s = mk(0.0, 0.0);
    for (int c = 0; c < nchunk; ++c) s = cadd(s, pc[(size_t)c * nvt * kSB + o]);
    D[o] = s;
  }
  __syncthreads();
  double2* cf = coef + (size_t)col * ldc;
  for (int o = threadIdx.x; o < k1 * kSB; o += kRed) cf[129 + o] = D[o];
  if (threadIdx.x < kSB * kSB) {
    const int p = threadIdx.x / kSB, l = threadIdx.x % kSB;
    double2 s = mk(0.0, 0.0);
    if (p < sb && l < sb) {
      s = D[(k1 + p) * kSB + l];
      for (int i = 0; i < k1; ++i) {  // s -= conj(C[i][p]) C[i][l]
        const double2 a = D[i * kSB + p], b = D[i * kSB + l];
        s.x -= a.x * b.x + a.y * b.y;
        s.y -= a.x * b.y - a.y * b.x;
      }
    }
    P[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double dsc[kSB];
  double2 Rs[kSB][kSB], X[kSB][kSB];
  for (int p = 0; p < kSB; ++p) {
    const double gpp = p < sb ? D[(k1 + p) * kSB + p].x : 0.0;
    dsc[p] = gpp > 0.0 ? sqrt(gpp) : 0.0;
    for (int q = 0; q < kSB; ++q) Rs[p][q] = X[p][q] = mk(0.0, 0.0);
  }
  int bk = sb;
  for (int l = 0; l < sb; ++l) {
    if (dsc[l] == 0.0) { bk = l; break; }
    double d = P[l * kSB + l].x / (dsc[l] * dsc[l]);
    for (int p = 0; p < l; ++p) d -= Rs[p][l].x * Rs[p][l].x + Rs[p][l].y * Rs[p][l].y;
    if (!(d > 1e-26)) { bk = l; break; }
    const double rll = sqrt(d);
    Rs[l][l] = mk(rll, 0.0);
    for (int q = l + 1; q < sb; ++q) {
      if (dsc[q] == 0.0) continue;
      const double sc = 1.0 / (dsc[l] * dsc[q]);
      double2 v = mk(P[l * kSB + q].x * sc, P[l * kSB + q].y * sc);
      for (int p = 0; p < l; ++p) {  // v -= conj(Rs[p][l]) Rs[p][q]
        const double2 a = Rs[p][l], b = Rs[p][q];
        v.x -= a.x * b.x + a.y * b.y;
        v.y -= a.x * b.y - a.y * b.x;
      }
      Rs[l][q] = mk(v.x / rll, v.y / rll);
    }
  }
  // inverse of the leading bk x bk block of Rs (upper triangular)
  for (int l = 0; l < bk; ++l) {
    X[l][l] = mk(1.0 / Rs[l][l].x, 0.0);
    for (int p = l - 1; p >= 0; --p) {
      double2 s = mk(0.0, 0.0);
      for (int q = p + 1; q <= l; ++q) cfma(s, Rs[p][q], X[q][l]);
      X[p][l] = mk(-s.x / Rs[p][p].x, -s.y / Rs[p][p].x);
    }
  }
  for (int p = 0; p < kSB; ++p)
    for (int q = 0; q < kSB; ++q) {
      const bool rv = p < bk && q >= p && q < sb;  // rows from bk on stay zero
      cf[p * kSB + q] = rv ? mk(Rs[p][q].x * dsc[q], Rs[p][q].y * dsc[q]) : mk(0.0, 0.0);
      const bool iv = q < bk && p <= q;
      cf[64 + p * kSB + q] = iv ? mk(X[p][q].x / dsc[p], X[p][q].y / dsc[p]) : mk(0.0, 0.0);
    }
  cf[128] = mk((double)bk, 0.0);
}

// Q = (Y - V C) R^{-1} in place of Y (V_{k1 + l}, l < sb), U positions per thread; grid
// (ceil(n / (256 U)), ncol).  The coefficients are the same for the whole workgroup.
template <int U>
__global__ __launch_bounds__(256) void k_bgs_update(double2* __restrict__ V, size_t vstride, int k1, int sb, int n,
                                                    const double2* __restrict__ coef, int ldc) {
  const int col = blockIdx.y;
  const double2* cf = coef + (size_t)col * ldc;
  const double2* C = cf + 129;
  const double2* Ri = cf + 64;
  int pos[U];
  bool in[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long q = ((long)blockIdx.x * U + u) * 256 + threadIdx.x;
    in[u] = q < n;
    pos[u] = in[u] ? (int)q : n - 1;
  }
  double2 y[U][kSB];
#pragma unroll
  for (int l = 0; l < kSB; ++l) {
    const double2* yp = V + (size_t)(k1 + min(l, sb - 1)) * vstride + (size_t)col * n;
#pragma unroll
    for (int u = 0; u < U; ++u) y[u][l] = yp[pos[u]];
  }
  for (int i = 0; i < k1; ++i) {
    const double2* vp = V + (size_t)i * vstride + (size_t)col * n;
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = vp[pos[u]];
#pragma unroll
    for (int l = 0; l < kSB; ++l) {
      const double2 c = C[i * kSB + l];
      const double2 mc = mk(-c.x, -c.y);
#pragma unroll
      for (int u = 0; u < U; ++u) cfma(y[u][l], v[u], mc);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (!in[u]) continue;
#pragma unroll
    for (int l = 0; l < kSB; ++l) {
      if (l >= sb) break;
      double2 q = mk(0.0, 0.0);
#pragma unroll
      for (int p = 0; p <= l; ++p) cfma(q, y[u][p], Ri[p * kSB + l]);
      V[(size_t)(k1 + l) * vstride + (size_t)col * n + pos[u]] = q;
    }
  }
}

constexpr int kUpdU = 2;

}  // namespace

// positions per wavefront of the inner-product pass: about 1024 workgroups over all columns,
// at least one batch of 16 positions
int bgs_positions_per_wave(int n, int ncol) {
  const long tot = (long)n * ncol;
  const long pw = (tot + (long)BW * 1024 - 1) / ((long)BW * 1024);
  return (int)std::max<long>(16, (pw + 15) / 16 * 16);
}

int bgs_chunks(int n, int ncol) {
  const int pw = bgs_positions_per_wave(n, ncol);
  return (int)(((long)n + (long)BW * pw - 1) / ((long)BW * pw));
}

size_t bgs_partial_elems(int n, int ncol) { return (size_t)ncol * bgs_chunks(n, ncol) * kSstepMaxBasis * kSB; }

hipError_t launch_bgs(double2* V, size_t vstride, int k1, int sb, int n, int ncol, double2* part, size_t part_elems,
                      double2* coef, int ldc, hipStream_t st) {
  const int nvt = k1 + sb;
  if (k1 < 1 || sb < 1 || sb > kSB || nvt > kSstepMaxBasis || n < 1 || ncol < 1 || ldc < kSstepCoefLd)
    return hipErrorInvalidValue;
  const int pw = bgs_positions_per_wave(n, ncol), nchunk = bgs_chunks(n, ncol);
  if ((size_t)ncol * nchunk * nvt * kSB > part_elems) return hipErrorInvalidValue;
  const dim3 gd(nchunk, ncol);
  switch ((nvt + 15) / 16) {
    case 1: k_bgs_dots<1><<<gd, 64 * BW, 0, st>>>(V, vstride, nvt, k1, sb, n, pw, part); break;
    case 2: k_bgs_dots<2><<<gd, 64 * BW, 0, st>>>(V, vstride, nvt, k1, sb, n, pw, part); break;
    case 3: k_bgs_dots<3><<<gd, 64 * BW, 0, st>>>(V, vstride, nvt, k1, sb, n, pw, part); break;
    default: k_bgs_dots<kTiles><<<gd, 64 * BW, 0, st>>>(V, vstride, nvt, k1, sb, n, pw, part); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_bgs_reduce<<<ncol, kRed, 0, st>>>(part, nchunk, nvt, k1, sb, coef, ldc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 gu((unsigned)(((long)n + 256 * kUpdU - 1) / (256 * kUpdU)), ncol);
  k_bgs_update<kUpdU><<<gu, 256, 0, st>>>(V, vstride, k1, sb, n, coef, ldc);
  return hipGetLastError();
}
