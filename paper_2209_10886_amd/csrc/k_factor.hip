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

// The same factorisation, blocked by panels of 16 columns (one workgroup per subdomain).  The
// column-by-column kernel above rewrites the whole (kl x kv) trailing window for every column;
// here a panel of 16 columns (rows [j0, j0 + 16 + kl)) is factored in LDS by one wavefront, and
// the trailing window is touched once per panel: its rows are permuted by the panel's composite
// interchange, the top 16 rows are solved with the panel's unit lower triangle (U12), and the rest
// receives the rank-16 update A22 -= L21 U12.  The panel is factored with its interchanges
// applied to whole panel rows (so L21 and L11 sit in the rows the trailing update needs); before
// it is written back, the interchanges that came after each column are undone on that column's
// multipliers, which restores the band convention (interchanges act on the trailing columns
// only).  Every element receives the same floating-point operations in the same order as in the
// column-by-column kernel (updates in increasing column order, the same complex fma, the same
// pivot choice), so the two give the same factors.
constexpr int BLU_NB = 16;
constexpr int BLU_THREADS = 256;
constexpr int BLU_CH = 64;  // trailing columns per staged chunk of U12
// row stride of the panel in LDS: 17 elements (272 bytes), so that lanes reading one column (one
// row each) fall on different banks (a stride of 16 elements puts every lane on the same banks)
constexpr int BLU_PS = BLU_NB + 1;

__device__ inline bool band_has(int r, int c, int kl, int kv) { return r - c <= kl && c - r <= kv; }

// (value, index) of a wavefront with the largest value, the smallest index among equal values;
// lanes without a candidate hold (-1, INT_MAX).  A DPP scan inside each row of 16 lanes (row_shr
// 1, 2, 4, 8: lane 15 of a row ends with the row's best), then the four row results.
template <int CTRL>
__device__ inline void argmax_step(double& v, int& i) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)0, (int)(unsigned)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)0xBFF00000, (int)(b >> 32), CTRL, 0xF, 0xF, false);  // -1.0
  const int oi = __builtin_amdgcn_update_dpp(0x7fffffff, i, CTRL, 0xF, 0xF, false);
  const double ov = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
__device__ inline int wave_argmax(double v, int i) {
  argmax_step<0x111>(v, i);  // row_shr:1
  argmax_step<0x112>(v, i);  // row_shr:2
  argmax_step<0x114>(v, i);  // row_shr:4
  argmax_step<0x118>(v, i);  // row_shr:8
  double bv = -1.0;
  int bi = 0x7fffffff;
#pragma unroll
  for (int rrow = 0; rrow < 4; ++rrow) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), 16 * rrow + 15);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * rrow + 15);
    const int ri = __builtin_amdgcn_readlane(i, 16 * rrow + 15);
    const double rv = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    if (rv > bv || (rv == bv && ri < bi)) {
      bv = rv;
      bi = ri;
    }
  }
  return bi;
}

__global__ __launch_bounds__(BLU_THREADS) void k_band_lu_blocked(double2* AB, int32_t* ipiv, int32_t* info, int n,
                                                                 int kl, int ku, int ldab) {
  extern __shared__ unsigned char smem_raw[];
  const int s = blockIdx.x;
  double2* ab = AB + (size_t)s * n * ldab;
  int32_t* ip = ipiv + (size_t)s * n;
  const int kv = kl + ku;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int prmax = BLU_NB + kl;
  double2* P = reinterpret_cast<double2*>(smem_raw);      // [prmax][BLU_PS] panel, row-major
  int* perm = reinterpret_cast<int*>(P + prmax * BLU_PS);  // [prmax] composite interchange of the panel rows
  int* jpv = perm + prmax;                                  // [BLU_NB] pivot offsets (-1: no interchange)
  int* sc = jpv + BLU_NB;                                   // [0] ju, [1] first zero pivot, [2] nD
  int* dst = sc + 4;                                        // [BLU_NB] rows below the panel receiving a panel row
  int* src = dst + BLU_NB;
  // [BLU_NB][BLU_CH] U12 rows of a chunk, at the next 16-byte boundary after the integer tables
  double2* Ush = reinterpret_cast<double2*>(
      reinterpret_cast<int*>(smem_raw) + (((src + BLU_NB - reinterpret_cast<int*>(smem_raw)) + 3) & ~3));
  auto A = [&](int r, int c) -> double2& { return ab[(size_t)c * ldab + kv + r - c]; };
  if (tid == 0) {
    sc[0] = 0;
    sc[1] = -1;
  }
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += BLU_NB) {
    const int nbj = min(BLU_NB, n - j0), prow = min(nbj + kl, n - j0);
    // 1. the panel into LDS (entries outside the band are zero)
    for (int t = tid; t < prow * BLU_NB; t += BLU_THREADS) {
      const int r = t / BLU_NB, c = t - r * BLU_NB;
      P[r * BLU_PS + c] = (c < nbj && band_has(j0 + r, j0 + c, kl, kv)) ? A(j0 + r, j0 + c) : mk(0.0, 0.0);
    }
    __syncthreads();
    // 2. factor the panel (wavefront 0), interchanges on whole panel rows
    if (w == 0) {
      int ju = sc[0], zero_at = sc[1];
      for (int q = lane; q < prow; q += 64) perm[q] = q;
      __builtin_amdgcn_wave_barrier();
      for (int k = 0; k < nbj; ++k) {
        const int j = j0 + k, km = min(kl, n - 1 - j);
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int r = lane; r <= km; r += 64) {
          const double v = cabs1(P[(k + r) * BLU_PS + k]);
          if (v > bv) { bv = v; bi = r; }
        }
        const int jp = wave_argmax(bv, bi);
        if (lane == 0) ip[j] = j + jp;
        const double2 piv = P[(k + jp) * BLU_PS + k];
        if (piv.x == 0.0 && piv.y == 0.0) {
          if (zero_at < 0) zero_at = j;
          if (lane == 0) jpv[k] = -1;
          __builtin_amdgcn_wave_barrier();
          continue;
        }
        ju = max(ju, min(j + ku + jp, n - 1));
        if (lane == 0) jpv[k] = jp;
        if (jp != 0) {
          if (lane < BLU_NB) {
            const double2 a = P[k * BLU_PS + lane], b = P[(k + jp) * BLU_PS + lane];
            P[k * BLU_PS + lane] = b;
            P[(k + jp) * BLU_PS + lane] = a;
          }
          if (lane == 0) {
            const int t = perm[k];
            perm[k] = perm[k + jp];
            perm[k + jp] = t;
          }
        }
        __builtin_amdgcn_wave_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (km > 0) {
          const double2 pinv = cdiv(mk(1.0, 0.0), P[k * BLU_PS + k]);
          for (int r = 1 + lane; r <= km; r += 64) P[(k + r) * BLU_PS + k] = cmul(P[(k + r) * BLU_PS + k], pinv);
          __builtin_amdgcn_wave_barrier();
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          // rank-1 update of the panel columns right of k: each lane holds its rows (at most
          // three: km <= 128 < 3 * 64) of the multiplier column and of the row-k entries in
          // registers; a zero entry of row k only adds exact zeros
          double2 nu[BLU_NB];
#pragma unroll
          for (int c = 0; c < BLU_NB; ++c) {
            const double2 u = P[k * BLU_PS + c];
            nu[c] = mk(-u.x, -u.y);
          }
#pragma unroll 1
          for (int t = 0; t < 3; ++t) {
            const int r = 1 + lane + 64 * t;
            if (r > km) continue;
            const double2 lr = P[(k + r) * BLU_PS + k];
            double2 row[BLU_NB];
#pragma unroll
            for (int c = 0; c < BLU_NB; ++c) row[c] = P[(k + r) * BLU_PS + c];
#pragma unroll
            for (int c = 0; c < BLU_NB; ++c)
              if (c > k && c < nbj) cfma(row[c], lr, nu[c]);
#pragma unroll
            for (int c = 0; c < BLU_NB; ++c) P[(k + r) * BLU_PS + c] = row[c];
          }
        }
        __builtin_amdgcn_wave_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
      if (lane == 0) {
        sc[0] = ju;
        sc[1] = zero_at;
        int nd = 0;  // rows below the panel that receive a panel row (the composite interchange)
        for (int q = nbj; q < prow; ++q)
          if (perm[q] != q) {
            dst[nd] = q;
            src[nd] = perm[q];
            ++nd;
          }
        sc[2] = nd;
      }
    }
    __syncthreads();
    const int JU = sc[0], nd = sc[2];
    const int c0 = j0 + nbj, ncol = JU - c0 + 1;
    // 3. trailing columns: permute their window rows, solve the top rows with L11 (one thread per column)
    for (int cc = tid; cc < ncol; cc += BLU_THREADS) {
      const int c = c0 + cc;
      double2 u[BLU_NB], v[BLU_NB];
#pragma unroll
      for (int k = 0; k < BLU_NB; ++k) {
        const int r = j0 + perm[min(k, prow - 1)];
        u[k] = (k < nbj && band_has(r, c, kl, kv)) ? A(r, c) : mk(0.0, 0.0);
      }
#pragma unroll
      for (int i = 0; i < BLU_NB; ++i) {
        const int r = j0 + src[min(i, BLU_NB - 1)];
        v[i] = (i < nd && band_has(r, c, kl, kv)) ? A(r, c) : mk(0.0, 0.0);
      }
#pragma unroll
      for (int i = 0; i < BLU_NB; ++i) {
        const int r = j0 + dst[min(i, BLU_NB - 1)];
        if (i < nd && band_has(r, c, kl, kv)) A(r, c) = v[i];
      }
      // (a zero pivot leaves a zero column below it, so its products add exact zeros)
      // column by column (each u[k] still receives its products in increasing i); the scheduling
      // barrier keeps the loads of L11 with their column instead of hoisting all of them
#pragma unroll
      for (int i = 0; i + 1 < BLU_NB; ++i) {
        const double2 nui = mk(-u[i].x, -u[i].y);
#pragma unroll
        for (int k = i + 1; k < BLU_NB; ++k) cfma(u[k], P[k * BLU_PS + i], nui);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int k = 0; k < BLU_NB; ++k)
        if (k < nbj && band_has(j0 + k, c, kl, kv)) A(j0 + k, c) = u[k];
    }
    __syncthreads();
    // 4. A22 -= L21 U12: rows [c0, c0 + kl) (64 per wavefront pass, coalesced along a column), the
    //    trailing columns in chunks of BLU_CH whose U12 rows are staged in LDS
    {
      const int nrow = min(kl, n - c0);
      const int groups = (nrow + 63) / 64;
      const int g = groups > 0 ? w % groups : 0, h = groups > 0 ? w / groups : 0, hs = max(1, 4 / max(groups, 1));
      const int rr = 64 * g + lane, r = c0 + rr;
      const bool active = groups > 0 && w < groups * hs;
      const bool live = active && rr < nrow;
      double2 l[BLU_NB];
#pragma unroll
      for (int k = 0; k < BLU_NB; ++k) l[k] = live ? P[(nbj + rr) * BLU_PS + k] : mk(0.0, 0.0);
      for (int cb = 0; cb < ncol; cb += BLU_CH) {
        const int nc = min(BLU_CH, ncol - cb);
        for (int t = tid; t < BLU_NB * BLU_CH; t += BLU_THREADS) {
          const int k = t / BLU_CH, cc = t - k * BLU_CH, c = c0 + cb + cc;
          Ush[t] = (k < nbj && cc < nc && band_has(j0 + k, c, kl, kv)) ? A(j0 + k, c) : mk(0.0, 0.0);
        }
        __syncthreads();
        // Branch-free: a zero multiplier or a zero U12 entry only adds an exact zero (the
        // column-by-column kernel skips those products; the factors differ at most in the sign of
        // zero entries).  Rows past the chunk read the zero padding of Ush.
        // Branch-free: a zero multiplier or a zero U12 entry only adds an exact zero (the
        // column-by-column kernel skips those products; the factors differ at most in the sign of
        // zero entries).  Batches of eight columns, the next batch's loads issued before the
        // current batch's products; columns past the chunk read the zero padding of Ush.
        if (active) {
          constexpr int BQ = 8;
          // loads are unconditional (row and column clamped into the window, which lies inside the
          // band), so the compiler can count them; only the stores are guarded
          const int rl = c0 + min(rr, nrow - 1);
          auto ld = [&](int cc, double2(&a)[BQ]) {
#pragma unroll
            for (int q = 0; q < BQ; ++q) a[q] = A(rl, c0 + cb + min(cc + q * hs, nc - 1));
          };
          auto upd = [&](int cc, double2(&a)[BQ]) {
            // k outermost: the eight columns' reads of U12 row k are in flight together and go to
            // eight independent accumulators (each element still takes its products in increasing k)
#pragma unroll
            for (int k = 0; k < BLU_NB; ++k) {
              double2 uk[BQ];
#pragma unroll
              for (int q = 0; q < BQ; ++q) uk[q] = Ush[k * BLU_CH + min(cc + q * hs, BLU_CH - 1)];
#pragma unroll
              for (int q = 0; q < BQ; ++q) cfma(a[q], l[k], mk(-uk[q].x, -uk[q].y));
              __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int q = 0; q < BQ; ++q) {
              const int cq = cc + q * hs;
              if (live && cq < nc) A(r, c0 + cb + cq) = a[q];
            }
          };
          double2 a0[BQ], a1[BQ];
          const int step = BQ * hs;
          int cc = h;
          if (cc < nc) ld(cc, a0);
          for (; cc < nc; cc += 2 * step) {
            if (cc + step < nc) ld(cc + step, a1);
            upd(cc, a0);
            if (cc + step >= nc) break;
            if (cc + 2 * step < nc) ld(cc + 2 * step, a0);
            upd(cc + step, a1);
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();  // every wavefront has its rows of L21
    // 5. restore the band convention on the panel's multipliers and write the panel back
    if (w == 0 && lane < nbj) {
      const int k = lane;
      for (int k2 = nbj - 1; k2 > k; --k2) {
        const int jp = jpv[k2];
        if (jp > 0) {
          const double2 a = P[k2 * BLU_PS + k], b = P[(k2 + jp) * BLU_PS + k];
          P[k2 * BLU_PS + k] = b;
          P[(k2 + jp) * BLU_PS + k] = a;
        }
      }
    }
    __syncthreads();
    for (int t = tid; t < prow * BLU_NB; t += BLU_THREADS) {
      const int r = t / BLU_NB, c = t - r * BLU_NB;
      if (c < nbj && band_has(j0 + r, j0 + c, kl, kv)) A(j0 + r, j0 + c) = P[r * BLU_PS + c];
    }
    __syncthreads();
  }
  if (tid == 0) info[s] = (sc[1] < 0) ? 0 : sc[1] + 1;
}

// One workgroup per (column block, subdomain).  Uses the block's slice of mf as scratch
// for the permuted multipliers before overwriting it with Mf.
template <int NB>
__global__ __launch_bounds__(256) void k_repack(Geom g, SolveLayout L, const double2* AB, const int32_t* ipiv,
                                                double2* MF, int16_t* PF, int32_t* PFLAG, double2* MB) {
  const int b = blockIdx.x, s = blockIdx.y;
  // kv: the band of U in the LU storage; kvb: the rows of U above a block that the backward window
  // holds (kv, or ku when no row was interchanged: U then has ku superdiagonals and the others are 0)
  const int n = g.nloc, kl = g.kl, kv = g.kv, ldab = g.ldab;
  const int wf = L.wf, wb = L.wb, kvb = solve_kvb(L);
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
  for (int q = tid; q < kvb; q += nt) {
    const int i = j0 - kvb + q;  // row of A above the block
    double2 urow[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double2 v = mk(0.0, 0.0);
      const int d = kv - kvb + q - c;  // storage row of U(i, j0 + c): kv + i - (j0 + c)
      if (i >= 0 && d >= 0 && j0 + c < n) v = ab[(size_t)(j0 + c) * ldab + d];
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
    MBX(c, kvb + r) = X[r][c];
  }
#undef MF
#undef MBX
}

__global__ void k_cast_c64(const double2* src, float2* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

}  // namespace

hipError_t launch_band_lu(const Geom& g, double2* ab, int32_t* ipiv, int32_t* info, int nsub, hipStream_t st,
                          bool blocked) {
  if (g.kl > 64 * MAX_ROWS_PER_LANE) return hipErrorInvalidValue;
  const size_t ints = ((size_t)(BLU_NB + g.kl) + 3 * BLU_NB + 4 + 3) & ~(size_t)3;  // perm, jpv, sc, dst, src
  const size_t shm = (size_t)(BLU_NB + g.kl) * BLU_PS * sizeof(double2) + ints * sizeof(int) +
                     (size_t)BLU_NB * BLU_CH * sizeof(double2);
  if (blocked && shm <= 64 * 1024 && g.kl < 3 * 64) {  // panel update: at most three rows per lane
    hipLaunchKernelGGL(k_band_lu_blocked, dim3(nsub), dim3(BLU_THREADS), shm, st, ab, ipiv, info, g.nloc, g.kl, g.ku,
                       g.ldab);
  } else {
    hipLaunchKernelGGL(k_band_lu, dim3(nsub), dim3(LU_THREADS), 0, st, ab, ipiv, info, g.nloc, g.kl, g.ku, g.ldab);
  }
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
