// Batched banded LU with partial pivoting of the local matrices, and its repack into
// the blocked layout used by the triangular solves.
//
// The paper solves each sub-problem with a sparse direct solver (Sec. 7).  Here each
// local matrix (n_loc = snx*sny unknowns, bandwidth kl = ku = snx in the natural
// ordering) is factored as P A = L U in LAPACK band storage with LAPACK's
// unblocked band algorithm (pivot = first index of max |re|+|im| in the column,
// U fill up to kl + ku superdiagonals, row interchanges applied to the trailing
// columns only, so L is a product of elementary transforms interleaved with the
// interchanges).
//
// Solve layout.  For a column block of nb columns starting at j0, the nb
// interchanges and eliminations act on the window of rows [j0, j0 + nb + kl).
// Moving every interchange to the right of the earlier eliminations (permuting
// those columns' multipliers) gives  T_blk = Lt^{-1} Pt  with Pt a permutation of
// the window and Lt unit lower trapezoidal.  With X = Lt11^{-1}:
//   y_top = X (Pt w)_top ,  w_rest <- (Pt w)_rest - Lt21 X (Pt w)_top
// so one block of the forward solve is a single (nb + kl) x nb matrix-vector
// product  Mf = [X ; -Lt21 X]  applied to the gathered window.  The backward solve
// uses, for the block of rows [j0, j0+nb), Y = U11^{-1} and the rows above it that
// couple to the block (U has kl + ku superdiagonals):  Mb = [-U_above Y ; Y],
// a (kl + ku + nb) x nb matrix.
#include "hbj_internal.h"

namespace {

constexpr int LU_THREADS = 512;
constexpr int MAX_ROWS_PER_LANE = 4;  // kl <= 256

__global__ __launch_bounds__(LU_THREADS) void k_band_lu(double2* AB, int32_t* ipiv, int32_t* info, int n, int kl,
                                                        int ku, int ldab) {
  const int s = blockIdx.x;
  double2* ab = AB + (size_t)s * n * ldab;
  int32_t* ip = ipiv + (size_t)s * n;
  const int kv = kl + ku;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  __shared__ double sv[LU_THREADS / 64];
  __shared__ int si[LU_THREADS / 64];
  int ju = 0, zero_at = -1;
  for (int j = 0; j < n; ++j) {
    const int km = min(kl, n - 1 - j);
    double2* colj = ab + (size_t)j * ldab + kv;  // colj[r] = A(j + r, j)
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int r = tid; r <= km; r += nt) {
      const double v = cabs1(colj[r]);
      if (v > bv) { bv = v; bi = r; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_down(bv, off);
      const int oi = __shfl_down(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { sv[wid] = bv; si[wid] = bi; }
    __syncthreads();
    double fv = sv[0];
    int jp = si[0];
    for (int w = 1; w < nw; ++w)
      if (sv[w] > fv || (sv[w] == fv && si[w] < jp)) { fv = sv[w]; jp = si[w]; }
    if (tid == 0) ip[j] = j + jp;
    const double2 piv = colj[jp];
    __syncthreads();
    if (piv.x == 0.0 && piv.y == 0.0) {
      if (zero_at < 0) zero_at = j;
      continue;
    }
    ju = max(ju, min(j + ku + jp, n - 1));
    if (jp != 0) {
      for (int c = j + tid; c <= ju; c += nt) {
        double2* col = ab + (size_t)c * ldab + kv - c;  // col[i] = A(i, c)
        const double2 a = col[j], b = col[j + jp];
        col[j] = b;
        col[j + jp] = a;
      }
      __syncthreads();
    }
    if (km > 0) {
      const double2 pinv = cdiv(mk(1.0, 0.0), colj[0]);
      for (int r = 1 + tid; r <= km; r += nt) colj[r] = cmul(colj[r], pinv);
      __syncthreads();
      double2 l[MAX_ROWS_PER_LANE];
#pragma unroll
      for (int t = 0; t < MAX_ROWS_PER_LANE; ++t) {
        const int r = 1 + lane + 64 * t;
        l[t] = (r <= km) ? colj[r] : mk(0.0, 0.0);
      }
      for (int c = j + 1 + wid; c <= ju; c += nw) {
        double2* col = ab + (size_t)c * ldab + kv - c;
        const double2 u = col[j];
        if (u.x != 0.0 || u.y != 0.0) {
          const double2 nu = mk(-u.x, -u.y);
#pragma unroll
          for (int t = 0; t < MAX_ROWS_PER_LANE; ++t) {
            const int r = 1 + lane + 64 * t;
            if (r <= km) {
              double2 a = col[j + r];
              cfma(a, l[t], nu);
              col[j + r] = a;
            }
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) info[s] = (zero_at < 0) ? 0 : zero_at + 1;
}

// One workgroup per (column block, subdomain).  Uses the block's slice of mf as scratch
// for the permuted multipliers before overwriting it with Mf.
template <int NB>
__global__ __launch_bounds__(256) void k_repack(Geom g, SolveLayout L, const double2* AB, const int32_t* ipiv,
                                                double2* MF, int16_t* PF, int32_t* PFLAG, double2* MB) {
  const int b = blockIdx.x, s = blockIdx.y;
  const int n = g.nloc, kl = g.kl, kv = g.kv, ldab = g.ldab;
  const int wf = L.wf, wb = L.wb;
  const double2* ab = AB + (size_t)s * n * ldab;
  const int32_t* ip = ipiv + (size_t)s * n;
  double2* mf = MF + (size_t)s * L.mf_per_sub + (size_t)b * NB * wf;  // tiled, see tile_index
  int16_t* pf = PF + (size_t)s * L.pf_per_sub + (size_t)b * wf;
  double2* mb = MB + (size_t)s * L.mb_per_sub + (size_t)b * NB * wb;  // tiled, see tile_index
  const int cgf = L.cgf, cgb = L.cgb;
#define MF(c, r) mf[tile_index((c), (r), wf, NB, cgf)]
#define MBX(c, q) mb[tile_index((c), (q), wb, NB, cgb)]
  const int j0 = b * NB;
  const int tid = threadIdx.x, nt = blockDim.x;

  __shared__ int piv[NB];
  __shared__ int16_t src[NB + 256 + 1];
  __shared__ double2 T[NB][NB + 1];
  __shared__ double2 X[NB][NB + 1];

  for (int c = tid; c < NB; c += nt) piv[c] = (j0 + c < n) ? ip[j0 + c] - j0 : c;
  for (int r = tid; r < wf; r += nt) src[r] = (int16_t)r;
  __syncthreads();
  // ---------------- forward ----------------
  if (tid == 0) {
    for (int c = 0; c < NB; ++c) {
      const int p = piv[c];
      const int16_t a = src[c];
      src[c] = src[p];
      src[p] = a;
    }
  }
  // multipliers of every column, unpermuted: window row r of column c holds A(j0 + r, j0 + c)
  for (int t = tid; t < NB * wf; t += nt) {
    const int c = t / wf, r = t - c * wf;
    double2 v = mk(0.0, 0.0);
    if (j0 + c < n && r > c && r <= c + kl && j0 + r < n) v = ab[(size_t)(j0 + c) * ldab + kv + (r - c)];
    MF(c, r) = v;
  }
  __syncthreads();
  for (int r = tid; r < wf; r += nt) pf[r] = src[r];
  if (tid == 0) {
    int ident = 1;
    for (int c = 0; c < NB; ++c) ident &= (piv[c] == c);
    PFLAG[(size_t)s * L.nblk + b] = ident;
  }
  // later interchanges act on the earlier columns' multipliers
  for (int c = tid; c < NB; c += nt) {
    for (int c2 = c + 1; c2 < NB; ++c2) {
      const int p = piv[c2];
      if (p != c2) {
        const double2 a = MF(c, c2);
        MF(c, c2) = MF(c, p);
        MF(c, p) = a;
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < NB * NB; t += nt) {
    const int c = t / NB, r = t - c * NB;
    T[r][c] = (r > c) ? MF(c, r) : mk(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // X = T^{-1} (unit lower), one column per thread
  for (int c = tid; c < NB; c += nt) {
    for (int r = 0; r < c; ++r) X[r][c] = mk(0.0, 0.0);
    X[c][c] = mk(1.0, 0.0);
    for (int r = c + 1; r < NB; ++r) {
      double2 acc = mk(0.0, 0.0);
      for (int k = c; k < r; ++k) cfma(acc, T[r][k], X[k][c]);
      X[r][c] = mk(-acc.x, -acc.y);
    }
  }
  __syncthreads();
  // rows below the triangle: -Lt21 X (each thread owns whole rows)
  for (int r = NB + tid; r < wf; r += nt) {
    double2 row[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) row[c] = MF(c, r);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double2 acc = mk(0.0, 0.0);
      for (int k = c; k < NB; ++k) cfma(acc, row[k], X[k][c]);
      MF(c, r) = mk(-acc.x, -acc.y);
    }
  }
  for (int t = tid; t < NB * NB; t += nt) {
    const int c = t / NB, r = t - c * NB;
    MF(c, r) = X[r][c];
  }
  __syncthreads();
  // ---------------- backward ----------------
  // U11 (upper, with diagonal); virtual columns beyond n are the identity
  for (int t = tid; t < NB * NB; t += nt) {
    const int c = t / NB, r = t - c * NB;
    double2 v = mk(0.0, 0.0);
    if (j0 + c >= n) v = mk(r == c ? 1.0 : 0.0, 0.0);
    else if (r <= c && c - r <= kv) v = ab[(size_t)(j0 + c) * ldab + kv + r - c];
    T[r][c] = v;
  }
  __syncthreads();
  for (int c = tid; c < NB; c += nt) {
    for (int r = c + 1; r < NB; ++r) X[r][c] = mk(0.0, 0.0);
    for (int r = c; r >= 0; --r) {
      double2 acc = mk(r == c ? 1.0 : 0.0, 0.0);
      for (int k = r + 1; k <= c; ++k) {
        const double2 p = cmul(T[r][k], X[k][c]);
        acc.x -= p.x;
        acc.y -= p.y;
      }
      X[r][c] = cdiv(acc, T[r][r]);
    }
  }
  __syncthreads();
  for (int q = tid; q < kv; q += nt) {
    const int i = j0 - kv + q;  // row of A above the block
    double2 urow[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double2 v = mk(0.0, 0.0);
      if (i >= 0 && c <= q && j0 + c < n) v = ab[(size_t)(j0 + c) * ldab + q - c];
      urow[c] = v;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double2 acc = mk(0.0, 0.0);
      for (int k = 0; k <= c; ++k) cfma(acc, urow[k], X[k][c]);
      MBX(c, q) = mk(-acc.x, -acc.y);
    }
  }
  for (int t = tid; t < NB * NB; t += nt) {
    const int c = t / NB, r = t - c * NB;
    MBX(c, kv + r) = X[r][c];
  }
#undef MF
#undef MBX
}

__global__ void k_cast_c64(const double2* src, float2* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

}  // namespace

hipError_t launch_band_lu(const Geom& g, double2* ab, int32_t* ipiv, int32_t* info, int nsub, hipStream_t st) {
  if (g.kl > 64 * MAX_ROWS_PER_LANE) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_band_lu, dim3(nsub), dim3(LU_THREADS), 0, st, ab, ipiv, info, g.nloc, g.kl, g.ku, g.ldab);
  return hipGetLastError();
}

hipError_t launch_repack(const Geom& g, const SolveLayout& L, const double2* ab, const int32_t* ipiv, double2* mf,
                         int16_t* pf, int32_t* pflag, double2* mb, int nsub, hipStream_t st) {
  if (L.nb != 16 || g.kl > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_repack<16>, dim3(L.nblk, nsub), dim3(256), 0, st, g, L, ab, ipiv, mf, pf, pflag, mb);
  return hipGetLastError();
}

hipError_t launch_cast_c64(const double2* src, float2* dst, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_c64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}
