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
constexpr int kTiles = kSstepMaxBasis / 16;

// Inner products D[i][l] = V_i^H Y_l (V_{k1 + l} = Y_l) for i < nvt = k1 + sb and l < kSB, per
// column, as partial sums over the positions of one workgroup and one part of its k-steps:
// part[(((col * nchunk + chunk) * KP + kp) * nvt + i) * kSB + l].
// Workgroup chunk takes positions [chunk cp, + cp) (cp a multiple of 64) of one column in batches
// of 64: each wavefront loads whole rows (one basis vector, 64 consecutive positions: 1 KB per
// load instruction) into a 16 NT x 64 LDS tile, the next batch's loads being in flight while the
// products of this one run.  The products are f64 MFMA 16x16x4 with the positions as the
// contraction index: A = the real or the imaginary parts of 16 basis vectors (lane (i, kk) holds
// row 16 t + i at position 4 q + kk of k-step q), B = the real parts of Y_0..Y_7 in its columns
// 0-7 and the imaginary parts in columns 8-15 (lane (c, kk)); then
// Re D = (Re V)^T (Re Y) + (Im V)^T (Im Y) and Im D = (Re V)^T (Im Y) - (Im V)^T (Re Y), column c
// and its partner c + 8 meeting by a lane exchange.  Wavefront w computes tile w % NT over the
// k-steps of part w / NT (NT = 3: one part, the fourth wavefront only loads).  Positions past the
// range are stored as zeros; rows past nvt hold copies of the last vector (never stored); the
// tile's 16-byte columns are XOR-swizzled by the row (conflict-free reads of 16 rows at one
// position).
template <int NT>
__global__ __launch_bounds__(256) void k_bgs_dots(const double2* __restrict__ V, size_t vstride, int nvt, int k1,
                                                  int sb, int n, int cp, double2* __restrict__ part) {
  constexpr int ROWS = 16 * NT, NL = ROWS / 4;
  constexpr int KP = (NT == 3) ? 1 : 4 / NT;  // parts of the 16 k-steps of a batch
  constexpr int KS = 16 / KP;                 // k-steps per wavefront and batch
  __shared__ double2 tile[ROWS * 64];
  const int chunk = blockIdx.x, col = blockIdx.y, nchunk = gridDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, kk = lane >> 4;
  const long p0l = (long)chunk * cp;
  const int p0 = (int)min(p0l, (long)n), p1 = (int)min(p0l + cp, (long)n);
  const double2* base = V + (size_t)col * n;
  double2 ld[NL];
  auto load = [&](int p) {
    const int pos = min(p + lane, n - 1);
#pragma unroll
    for (int j = 0; j < NL; ++j) ld[j] = base[(size_t)min(wv + 4 * j, nvt - 1) * vstride + pos];
  };
  auto at = [](int row, int c) { return row * 64 + (c ^ (row & 15)); };
  const int mt = (NT == 3) ? wv : wv % NT;
  const int kp = (NT == 3) ? 0 : wv / NT;
  const bool active = mt < NT;
  const int l = r16 & 7;
  const bool take_re = r16 < 8, lok = l < sb;
  const int arow = 16 * (active ? mt : 0) + r16, brow = k1 + (lok ? l : 0);
  d4v a1 = d4v{0.0, 0.0, 0.0, 0.0}, a2 = d4v{0.0, 0.0, 0.0, 0.0};
  if (p0 < p1) load(p0);
  for (int p = p0; p < p1; p += 64) {
    __syncthreads();  // the products of the previous batch have read the tile
    const bool in = p + lane < p1;
#pragma unroll
    for (int j = 0; j < NL; ++j) tile[at(wv + 4 * j, lane)] = in ? ld[j] : mk(0.0, 0.0);
    __syncthreads();
    if (p + 64 < p1) load(p + 64);
    if (active) {
#pragma unroll
      for (int qq = 0; qq < KS; ++qq) {
        const int c = 4 * (kp * KS + qq) + kk;
        const double2 av = tile[at(arow, c)];
        const double2 bv = tile[at(brow, c)];
        const double b = lok ? (take_re ? bv.x : bv.y) : 0.0;
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, b, a1, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, b, a2, 0, 0, 0);
      }
    }
  }
  if (!active) return;
  // accumulator register r of lane (c, kk) holds row kk + 4 r, column c of the 16 x 16 tile
  double2* out = part + (((size_t)col * nchunk + chunk) * KP + kp) * nvt * kSB;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double x1 = a1[r], x2 = a2[r];
    const double y1 = __shfl_xor(x1, 8), y2 = __shfl_xor(x2, 8);  // column c + 8 of the same row
    const int i = 16 * mt + kk + 4 * r;
    if (r16 < 8 && i < nvt) out[i * kSB + r16] = mk(x1 + y2, y1 - x2);
  }
}

// Per column: D = the sum of the partials in a fixed order, C = D[0..k1), the Gram matrix
// G[p][l] = D[k1 + p][l] = Y_p^H Y_l, P = G - C^H C, and the Cholesky factor R (upper, P = R^H R)
// of P scaled by 1/sqrt(G_pp G_ll), scaled back; R^{-1} alongside.  Record of column col at
// coef + col ldc: R[p][l] at p kSB + l, R^{-1} at 64 + p kSB + l, at 128 the index b of the first
// pivot that failed (sb if none) as a double, and C[i][l] at 129 + i kSB + l.  A pivot fails when
// y_{b+1} has (relative to its norm) no component beyond 1e-13 outside the span of the basis and
// the earlier new vectors, or is zero: R's rows from b on are then zero, and so are the columns of
// R^{-1} from b on, which makes those vectors of Q zero.  The factorisation is right-looking, one
// thread per entry of the 8 x 8 matrix; the inverse one thread per column.
constexpr int kRed = 256;
__global__ __launch_bounds__(kRed) void k_bgs_reduce(const double2* __restrict__ part, int nset, int nvt, int k1,
                                                     int sb, double2* __restrict__ coef, int ldc) {
  const int col = blockIdx.x, tid = threadIdx.x;
  __shared__ double2 D[kSstepMaxBasis * kSB];
  __shared__ double2 P[kSB][kSB], R[kSB][kSB], X[kSB][kSB];
  __shared__ double dsc[kSB];
  __shared__ int bk_s;
  const double2* pc = part + (size_t)col * nset * nvt * kSB;
  for (int o = tid; o < nvt * kSB; o += kRed) {
    double2 s0 = mk(0.0, 0.0), s1 = mk(0.0, 0.0), s2 = mk(0.0, 0.0), s3 = mk(0.0, 0.0);
    int c = 0;
    for (; c + 4 <= nset; c += 4) {
      s0 = cadd(s0, pc[(size_t)c * nvt * kSB + o]);
      s1 = cadd(s1, pc[(size_t)(c + 1) * nvt * kSB + o]);
      s2 = cadd(s2, pc[(size_t)(c + 2) * nvt * kSB + o]);
      s3 = cadd(s3, pc[(size_t)(c + 3) * nvt * kSB + o]);
    }
    for (; c < nset; ++c) s0 = cadd(s0, pc[(size_t)c * nvt * kSB + o]);
    D[o] = cadd(cadd(s0, s1), cadd(s2, s3));
  }
  if (tid == 0) bk_s = sb;
  __syncthreads();
  double2* cf = coef + (size_t)col * ldc;
  for (int o = tid; o < k1 * kSB; o += kRed) cf[129 + o] = D[o];
  const int pr = tid / kSB, pl = tid % kSB;  // entry of the 8 x 8 matrices (tid < 64)
  if (tid < kSB) {
    const double g = tid < sb ? D[(k1 + tid) * kSB + tid].x : 0.0;
    dsc[tid] = g > 0.0 ? sqrt(g) : 0.0;
  }
  __syncthreads();
  if (tid < kSB * kSB) {
    double2 s = mk(0.0, 0.0);
    if (pr < sb && pl < sb && dsc[pr] > 0.0 && dsc[pl] > 0.0) {
      s = D[(k1 + pr) * kSB + pl];
      for (int i = 0; i < k1; ++i) {  // s -= conj(C[i][pr]) C[i][pl]
        const double2 a = D[i * kSB + pr], b = D[i * kSB + pl];
        s.x -= a.x * b.x + a.y * b.y;
        s.y -= a.x * b.y - a.y * b.x;
      }
      const double sc = 1.0 / (dsc[pr] * dsc[pl]);
      s = mk(s.x * sc, s.y * sc);
    }
    P[pr][pl] = s;
    R[pr][pl] = X[pr][pl] = mk(0.0, 0.0);
  }
  __syncthreads();
  for (int l = 0; l < sb; ++l) {
    if (tid == 0) {
      const double d = P[l][l].x;
      if (dsc[l] == 0.0 || !(d > 1e-26)) bk_s = l;
      else R[l][l] = mk(sqrt(d), 0.0);
    }
    __syncthreads();
    if (bk_s <= l) break;
    if (tid < kSB && tid > l && tid < sb) {
      const double2 v = P[l][tid];
      R[l][tid] = mk(v.x / R[l][l].x, v.y / R[l][l].x);
    }
    __syncthreads();
    if (tid < kSB * kSB && pr > l && pl >= pr && pl < sb) {  // trailing update: P -= conj(R[l][pr]) R[l][pl]
      const double2 a = R[l][pr], b = R[l][pl];
      P[pr][pl].x -= a.x * b.x + a.y * b.y;
      P[pr][pl].y -= a.x * b.y - a.y * b.x;
    }
    __syncthreads();
  }
  const int bk = bk_s;
  if (tid < bk) {  // column tid of the inverse of the leading bk x bk block
    const int c = tid;
    X[c][c] = mk(1.0 / R[c][c].x, 0.0);
    for (int p = c - 1; p >= 0; --p) {
      double2 s = mk(0.0, 0.0);
      for (int q = p + 1; q <= c; ++q) cfma(s, R[p][q], X[q][c]);
      X[p][c] = mk(-s.x / R[p][p].x, -s.y / R[p][p].x);
    }
  }
  __syncthreads();
  if (tid < kSB * kSB) {
    const bool rv = pr < bk && pl >= pr && pl < sb;  // rows from bk on stay zero
    cf[tid] = rv ? mk(R[pr][pl].x * dsc[pl], R[pr][pl].y * dsc[pl]) : mk(0.0, 0.0);
    const bool iv = pl < bk && pr <= pl;
    cf[64 + tid] = iv ? mk(X[pr][pl].x / dsc[pr], X[pr][pl].y / dsc[pr]) : mk(0.0, 0.0);
  }
  if (tid == 0) cf[128] = mk((double)bk, 0.0);
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

// positions per workgroup of the inner-product pass: a multiple of 64 giving about as many
// workgroups over all columns as are resident at once (the LDS tile of NT x 16 KB allows two per
// compute unit with four tiles, three with three, four or more with fewer)
namespace {
int bgs_target_wgs(int nt) { return nt >= 4 ? 512 : nt == 3 ? 768 : 1024; }
int bgs_kparts(int nt) { return nt == 3 ? 1 : 4 / nt; }
}  // namespace

int bgs_positions_per_wg(int n, int ncol, int wgs) {
  const long tot = (long)n * ncol;
  const long cp = (tot + wgs - 1) / wgs;
  return (int)std::max<long>(64, (cp + 63) / 64 * 64);
}

int bgs_chunks(int n, int ncol, int wgs) {
  const int cp = bgs_positions_per_wg(n, ncol, wgs);
  return (int)(((long)n + cp - 1) / cp);
}

size_t bgs_partial_elems(int n, int ncol) {
  return (size_t)ncol * bgs_chunks(n, ncol, bgs_target_wgs(1)) * bgs_kparts(1) * kSstepMaxBasis * kSB;
}

hipError_t launch_bgs(double2* V, size_t vstride, int k1, int sb, int n, int ncol, double2* part, size_t part_elems,
                      double2* coef, int ldc, hipStream_t st) {
  const int nvt = k1 + sb;
  if (k1 < 1 || sb < 1 || sb > kSB || nvt > kSstepMaxBasis || n < 1 || ncol < 1 || ldc < kSstepCoefLd)
    return hipErrorInvalidValue;
  const int nt = (nvt + 15) / 16, wgs = bgs_target_wgs(nt), kp = bgs_kparts(nt);
  const int cp = bgs_positions_per_wg(n, ncol, wgs), nchunk = bgs_chunks(n, ncol, wgs);
  if ((size_t)ncol * nchunk * kp * nvt * kSB > part_elems) return hipErrorInvalidValue;
  const dim3 gd(nchunk, ncol);
  switch (nt) {
    case 1: k_bgs_dots<1><<<gd, 256, 0, st>>>(V, vstride, nvt, k1, sb, n, cp, part); break;
    case 2: k_bgs_dots<2><<<gd, 256, 0, st>>>(V, vstride, nvt, k1, sb, n, cp, part); break;
    case 3: k_bgs_dots<3><<<gd, 256, 0, st>>>(V, vstride, nvt, k1, sb, n, cp, part); break;
    default: k_bgs_dots<kTiles><<<gd, 256, 0, st>>>(V, vstride, nvt, k1, sb, n, cp, part); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_bgs_reduce<<<ncol, kRed, 0, st>>>(part, nchunk * kp, nvt, k1, sb, coef, ldc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 gu((unsigned)(((long)n + 256 * kUpdU - 1) / (256 * kUpdU)), ncol);
  k_bgs_update<kUpdU><<<gu, 256, 0, st>>>(V, vstride, k1, sb, n, coef, ldc);
  return hipGetLastError();
}
