// Dense local scattering operators applied to many right-hand sides at once:
//   OUT_s (rows x R) = T_s[rows, :] (L x L, masked rows) * G_s (L x R)
// a complex matrix product per subdomain, on MFMA.  Complex products use three real products
// per k-step (Gauss's product: Re = Ar Br - Ai Bi, Im = (Ar + Ai)(Br + Bi) - Ar Br - Ai Bi)
// instead of four.
//
// Operand layouts of the 16x16x4 MFMA on gfx950 (lane l, k = l / 16):
//   A[i][k] at lane i + 16 k, B[k][j] at lane j + 16 k;
//   f64: D[i][j] in lane j + 16 (i % 4), register i / 4;
//   f32: D[i][j] in lane j + 16 (i / 4), register i % 4.
#include <type_traits>

#include "hbj_internal.h"

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// G[j][col][r] = incoming datum of subdomain subs[j] at local interface position col, column r
// With coef, every datum is scaled by inj of its position: the incoming data in the form the
// lifting matrices W_s take for the reconstruction (x_col = W_s[.][col] inj_col).  GT: complex128,
// or complex64 for the products on f32 MFMA (which round every operand to float anyway).
// A transpose through LDS: workgroup (chunk, j, rb) reads kGP consecutive positions of 64 columns
// (right-hand sides) with the positions fastest (a face's positions are consecutive in gin) and
// writes them with the columns fastest (a row of G), so that both sides are contiguous runs.
// Columns past nrhs, and positions on faces without a neighbour, are zeros.
constexpr int kGP = 32;  // positions per gather workgroup
template <typename GT>
__global__ __launch_bounds__(256) void k_gather_incoming(Geom g, const int32_t* subs, const FaceTab* ft,
                                                         const double2* gin, int nrhs, int rpad, GT* G,
                                                         const IfCoef* coef) {
  const int j = blockIdx.y;
  const int s = subs ? subs[j] : j;
  const FaceTab F = ft[s];
  const int L = local_if_len(g);
  const int c0 = blockIdx.x * kGP, r0 = blockIdx.z * 64;
  __shared__ GT tile[kGP][65];
#pragma unroll
  for (int k = 0; k < kGP * 64 / 256; ++k) {
    const int idx = threadIdx.x + 256 * k;
    const int c = idx % kGP, r = idx / kGP;
    const int col = c0 + c, rr = r0 + r;
    double2 v = mk(0.0, 0.0);
    if (col < L && rr < nrhs) {
      int f, ee;
      local_if_face(g, col, &f, &ee);
      const int io = pick4(F.in_off, f);
      if (io >= 0) {
        v = gin[(size_t)rr * g.nif + io + ee];
        if (coef) v = cmul(coef[io + ee].inj, v);
      }
    }
    tile[c][r] = to_c<GT>(v);
  }
  __syncthreads();
  const size_t n = (size_t)L * rpad;
#pragma unroll
  for (int k = 0; k < kGP * 64 / 256; ++k) {
    const int idx = threadIdx.x + 256 * k;
    const int c = idx / 64, r = idx % 64;
    const int col = c0 + c, rr = r0 + r;
    if (col < L && rr < rpad) G[(size_t)j * n + (size_t)col * rpad + rr] = tile[c][r];
  }
}

// Gathered tiles of a whole preconditioner pass at its start: job q copies interface position
// pos[q] of the 64 columns [r0, r0 + 64) to tile entries dst[q] + r (element type GT), the same
// LDS transpose as k_gather_incoming (the jobs of one face are consecutive positions).
template <typename GT>
__global__ __launch_bounds__(256) void k_pregather(const int64_t* __restrict__ dst, const int32_t* __restrict__ pos,
                                                   int njobs, const double2* gin, int nif, int nrhs, int rpad,
                                                   GT* tiles) {
  const int q0 = blockIdx.x * kGP, r0 = blockIdx.y * 64;
  __shared__ GT tile[kGP][65];
#pragma unroll
  for (int k = 0; k < kGP * 64 / 256; ++k) {
    const int idx = threadIdx.x + 256 * k;
    const int c = idx % kGP, r = idx / kGP;
    const int q = q0 + c, rr = r0 + r;
    double2 v = mk(0.0, 0.0);
    if (q < njobs && rr < nrhs) v = gin[(size_t)rr * nif + pos[q]];
    tile[c][r] = to_c<GT>(v);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kGP * 64 / 256; ++k) {
    const int idx = threadIdx.x + 256 * k;
    const int c = idx / 64, r = idx % 64;
    const int q = q0 + c, rr = r0 + r;
    if (q < njobs && rr < rpad) tiles[dst[q] + rr] = tile[c][r];
  }
}

__device__ inline int masked_row_mm(const Geom& g, int mask, int r) {
  for (int f = 0; f < 4; ++f) {
    if (!((mask >> f) & 1)) continue;
    const int len = face_len(g, f);
    if (r < len) return face_off(g, f) + r;
    r -= len;
  }
  return -1;
}

template <typename M> struct MfmaAcc;
template <> struct MfmaAcc<double> {
  typedef d4v T;
  static __device__ inline T mma(double a, double b, T c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row_of(int lane, int reg) { return (lane >> 4) + 4 * reg; }
};
template <> struct MfmaAcc<float> {
  typedef f4v T;
  static __device__ inline T mma(float a, float b, T c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row_of(int lane, int reg) { return 4 * (lane >> 4) + reg; }
};

constexpr int TB = 4;  // 16-column right-hand-side blocks per wavefront (64 right-hand sides)
constexpr int KW = 4;  // wavefronts splitting the k range of one tile (KWT, the template value, may be 8)

// grid: (ceil(masked rows / 16), nsub, ceil(R / 64)).  One 16-row x 64-column output tile per
// workgroup; wavefront w takes every KW-th group of 4 columns of each existing face, and the four
// partial tiles are summed in LDS.  Each wavefront issues the loads of KB k-steps (column indices
// clamped into the face, out-of-range steps zeroed after the load) before their MFMAs, which go to
// eight independent accumulators.  The B operands (lane (j, k) of a k-step: right-hand side j at
// the step's position k) come either from the gathered tiles G ([nsub][L][rpad], element type C:
// right-hand sides contiguous) or, DIRECT, straight from the interface vector gin ([R][nif],
// complex128: positions contiguous), where the products on f32 MFMA round them to float at use.
// With NS = 2 the workgroup has two groups of KW wavefronts, each taking half of the right-hand-side
// blocks (two wavefronts per SIMD, so one's MFMAs overlap the other's loads; the A operands are
// loaded by both groups).  KB, NS and the source of B are chosen by the autotuner.
// RING > 0: instead of batches of KB k-steps per face, the wavefront walks its k-steps over all
// faces as one sequence (padded to a multiple of RING with masked steps) through a register ring of
// RING k-steps: the loads of step q + RING are issued right after the products of step q, so RING
// steps of loads are always in flight and a wait covers one step's loads only.
// XO: the workgroups take their (row tile, subdomain, right-hand-side tile) in XCD order, so that
// the 16 row tiles of a subdomain, which all read its incoming data, run on one XCD.
// KWT: wavefronts splitting the k range (4; 8 with NS = 1: eight wavefronts, each a 16-row x
// 64-column tile over an eighth of the columns, so that each A operand is loaded once).
template <typename C, typename M, int KB, bool DIRECT, int NS, int RING = 0, bool XO = false, int KWT = KW>
__global__ __launch_bounds__(64 * KWT * NS) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_scatter_mm(Geom g, const int32_t* subs, int mask, const FaceTab* ft,
                                                        const C* __restrict__ T,
                                                        const std::conditional_t<DIRECT, double2, C>* __restrict__ B,
                                                        int nrhs, int rpad, SolveIO io) {
  typedef std::conditional_t<DIRECT, double2, C> BT;
  typedef MfmaAcc<M> A;
  typedef typename A::T V4;
  constexpr int TW = TB / NS;  // right-hand-side blocks per wavefront
  int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  if constexpr (XO) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = xcd_tile(bx + gx * (by + gy * bz), gx * gy * gridDim.z);
    bx = t % gx;
    by = (t / gx) % gy;
    bz = t / (gx * gy);
  }
  const int j = by;
  const int s = subs[j];
  const FaceTab F = ft[s];
  const int L = local_if_len(g);
  const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) % KWT, grp = (threadIdx.x >> 6) / KWT;
  const int i = lane & 15, k = lane >> 4;
  const int mrow = masked_row_mm(g, mask, bx * 16 + i);  // this lane's A row
  const M amask = mrow >= 0 ? (M)1 : (M)0;
  const int rb0 = bz * 16 * TB;  // first right-hand side of the workgroup's tile
  const int tb0 = grp * TW;               // first right-hand-side block of this wavefront
  const C* Ts = T + (size_t)s * t_per_sub(g) + t_index(L, mrow < 0 ? 0 : mrow, 0);
  // right-hand sides of this lane's B operands, clamped to the last one (columns past nrhs only
  // feed output columns that are dropped); B element (rhs, col) at bface[jr + col * cs]
  const long cs = DIRECT ? 1 : rpad;
  long jr[TW];
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    const long r = min(rb0 + 16 * (tb0 + t) + i, nrhs - 1);
    jr[t] = DIRECT ? r * g.nif : (long)j * L * rpad + r;
  }
  // the epilogue's outputs, with their base values loaded before the k loop (wavefronts of group 0:
  // pair p = w + KWT n is block t = p / 4, register reg = p % 4); an output that is not stored
  // loads the interface vector's first entry instead (every load in bounds and unconditional)
  constexpr int NP = (TB * 4 + KWT - 1) / KWT;
  size_t opos[NP];
  double2 obase[NP];
  int oslot[NP];  // chained steps: the output's slot in the next step's tile (-1: none)
  if (grp == 0) {
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const int p = w + KWT * n;
      const int reg = p & 3;
      const int row = masked_row_mm(g, mask, bx * 16 + A::row_of(lane, reg));
      const int rhs = rb0 + 16 * (p >> 2) + (lane & 15);
      int rf = 0, re = 0;
      if (row >= 0) local_if_face(g, row, &rf, &re);
      const int oo = pick4(F.out_off, rf);
      const bool ok = p < TB * 4 && row >= 0 && rhs < nrhs && oo >= 0;
      opos[n] = ok ? (size_t)rhs * g.nif + oo + re : ~(size_t)0;
      obase[n] = io.tr_base ? io.tr_base[ok ? opos[n] : 0] : mk(0.0, 0.0);
      if (io.tr_sub) obase[n] = csub(obase[n], io.tr_sub[ok ? opos[n] : 0]);
      oslot[n] = (io.cmap && ok) ? io.cmap[oo + re] : -1;
    }
  }
  // complex products with three real MFMAs per k-step: cr += Ar Br, ci += Ai Bi,
  // c3 += (Ar + Ai)(Br + Bi), then Re = cr - ci and Im = c3 - cr - ci (Gauss's product; measured
  // against four products (Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br, kept below for reference):
  // complex128 operator 592 -> 514 us, complex64 sweep steps 18.2 -> 17.5 us for 64 sources at
  // 2048^2, the same iterations)
  constexpr bool K3 = true;
  V4 cr[TW], ci[TW], c3[TW];
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    cr[t] = V4{0, 0, 0, 0};
    ci[t] = V4{0, 0, 0, 0};
    c3[t] = V4{0, 0, 0, 0};
  }
  const int present[4] = {F.in_off[0] >= 0, F.in_off[1] >= 0, F.in_off[2] >= 0, F.in_off[3] >= 0};
  if constexpr (RING > 0) {
    // one flat sequence of k-steps over all L columns: step m covers columns 4 (KWT m + w) + k, each
    // lane finds its own face with three compares, and columns past L or on faces without data load
    // column 0 (every load in bounds) and enter the products as zero (by select: the operator's
    // entries there are never read otherwise)
    const int b1 = g.sny, b2 = 2 * g.sny, b3 = 2 * g.sny + g.snx;
    const int pm = present[0] | present[1] << 1 | present[2] << 2 | present[3] << 3;
    // offsets of the incoming data of each face in gin (DIRECT): position c of face f at fo_f + c
    const int fo0 = DIRECT ? F.in_off[0] : 0, fo1 = DIRECT ? F.in_off[1] - b1 : 0;
    const int fo2 = DIRECT ? F.in_off[2] - b2 : 0, fo3 = DIRECT ? F.in_off[3] - b3 : 0;
    const int ics = (int)cs;
    const int nst = (L + 4 * KWT - 1) / (4 * KWT);
    const int nsp = (nst + RING - 1) / RING * RING;
    C tv[RING];
    BT gv[RING][TW];
    bool live[RING];
    auto issue = [&](int m, int d) {
      const int col = 4 * (KWT * m + w) + k;
      const bool c1 = col >= b1, c2 = col >= b2, c3 = col >= b3;
      const int f = (int)c1 + (int)c2 + (int)c3;
      const bool ok = (col < L) & ((pm >> f) & 1);
      // the face's offset by 0/1 products (a select chain here becomes an indexed table in memory)
      const int fo = fo0 + (int)c1 * (fo1 - fo0) + (int)c2 * (fo2 - fo1) + (int)c3 * (fo3 - fo2);
      const int cc = ok ? col : 0;
      const int off = ok ? fo + cc * ics : 0;
      live[d] = ok;
      tv[d] = Ts[(size_t)cc * kTR];
#pragma unroll
      for (int t = 0; t < TW; ++t) gv[d][t] = B[jr[t] + off];
    };
    auto consume = [&](int d) {
      const bool ok = live[d] && mrow >= 0;
      const M ar = ok ? (M)tv[d].x : (M)0, ai = ok ? (M)tv[d].y : (M)0;
      if constexpr (K3) {
        const M as = ar + ai;
#pragma unroll
        for (int t = 0; t < TW; ++t) {
          const M br = (M)gv[d][t].x, bi = (M)gv[d][t].y;
          cr[t] = A::mma(ar, br, cr[t]);
          ci[t] = A::mma(ai, bi, ci[t]);
          c3[t] = A::mma(as, br + bi, c3[t]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < TW; ++t) {
          const M br = (M)gv[d][t].x, bi = (M)gv[d][t].y;
          cr[t] = A::mma(ar, br, cr[t]);
          ci[t] = A::mma(ar, bi, ci[t]);
        }
#pragma unroll
        for (int t = 0; t < TW; ++t) {
          const M br = (M)gv[d][t].x, bi = (M)gv[d][t].y;
          cr[t] = A::mma(-ai, bi, cr[t]);
          ci[t] = A::mma(ai, br, ci[t]);
        }
      }
    };
#pragma unroll
    for (int d = 0; d < RING; ++d) issue(d, d);
    for (int m0 = 0; m0 < nsp; m0 += RING) {
#pragma unroll
      for (int d = 0; d < RING; ++d) {
        consume(d);
        issue(m0 + d + RING, d);
      }
    }
  } else {
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if (!present[f]) continue;
    const int c0 = face_off(g, f), c1 = c0 + face_len(g, f);
    const long fo = DIRECT ? (long)pick4(F.in_off, f) - c0 : 0;  // gin[rhs * nif + fo + col]
    // this wavefront's k-steps: c0 + 4 (w + KWT q), KB of them per batch
    for (int c = c0 + 4 * w; c < c1; c += 4 * KWT * KB) {
      C tv[KB];
      BT gv[KB][TW];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const int col = c + 4 * KWT * b + k;
        const int cc = col < c1 ? col : c1 - 1;
        tv[b] = Ts[(size_t)cc * kTR];
#pragma unroll
        for (int t = 0; t < TW; ++t) gv[b][t] = B[jr[t] + fo + (long)cc * cs];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the whole batch of loads ahead of the MFMAs
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const M ok = (c + 4 * KWT * b + k < c1) ? amask : (M)0;
        const M ar = (M)tv[b].x * ok, ai = (M)tv[b].y * ok;
        if constexpr (K3) {
          const M as = ar + ai;
#pragma unroll
          for (int t = 0; t < TW; ++t) {
            const M br = (M)gv[b][t].x, bi = (M)gv[b][t].y;
            cr[t] = A::mma(ar, br, cr[t]);
            ci[t] = A::mma(ai, bi, ci[t]);
            c3[t] = A::mma(as, br + bi, c3[t]);
          }
        } else {
#pragma unroll
          for (int t = 0; t < TW; ++t) {
            const M br = (M)gv[b][t].x, bi = (M)gv[b][t].y;
            cr[t] = A::mma(ar, br, cr[t]);
            ci[t] = A::mma(ar, bi, ci[t]);
            cr[t] = A::mma(-ai, bi, cr[t]);
            ci[t] = A::mma(ai, br, ci[t]);
          }
        }
      }
    }
  }
  }
  // sum the KWT partial tiles: wavefront w of group 0 finishes the (block t, register reg) pairs
  // p = w, w + KWT, ... of the 16 (t = p / 4, reg = p % 4)
  __shared__ M red[KWT][TB][2][4][64];
#pragma unroll
  for (int t = 0; t < TW; ++t)
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) {
      red[w][tb0 + t][0][reg][lane] = K3 ? cr[t][reg] - ci[t][reg] : cr[t][reg];
      red[w][tb0 + t][1][reg][lane] = K3 ? c3[t][reg] - cr[t][reg] - ci[t][reg] : ci[t][reg];
    }
  __syncthreads();
  if (grp != 0) return;
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    const int p = w + KWT * n;
    if (p >= TB * 4) break;  // uniform
    const int t = p >> 2, reg = p & 3;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int q = 0; q < KWT; ++q) {
      sr += (double)red[q][t][0][reg][lane];
      si += (double)red[q][t][1][reg][lane];
    }
    if (opos[n] == ~(size_t)0) continue;
    double2 base = obase[n];
    base.x += io.tr_sign * sr;
    base.y += io.tr_sign * si;
    io.tr_dst[opos[n]] = base;
    if (oslot[n] >= 0)
      ((C*)io.ctile)[(size_t)oslot[n] * io.crpad + rb0 + 16 * (p >> 2) + (lane & 15)] = to_c<C>(base);
  }
}

// Reconstruction for many right-hand sides on MFMA (complex128 on f64 16x16x4):
//   U_s[p][r] = sum_col W_s[p][col] Gs[col][r]   (Gs: incoming data scaled by inj)
// and u[r] at node p of subdomain s = (nz ? u : 0) + U_s[p][r].  Workgroup = 4 wavefronts, each a
// 16-node x 64-RHS tile (4 blocks of 16 RHS) over the whole k range; the loads of KB k-steps are
// issued (clamped, unconditional) before their MFMAs.
template <int KB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_recon_mm(
    Geom g, const double2* __restrict__ W, const double2* __restrict__ Gs, int nrhs, int rpad, const int32_t* nz,
    double2* u) {
  typedef MfmaAcc<double> A;
  typedef A::T V4;
  const int s = blockIdx.y;
  const int L = local_if_len(g);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, k = lane >> 4;
  const int p0 = (blockIdx.x * 4 + w) * 16;
  const int prow = min(p0 + i, g.nloc - 1);  // this lane's A row (clamped; tail rows are not stored)
  const int rb0 = blockIdx.z * 16 * TB;
  const double2* Wr = W + ((size_t)s * g.nloc + prow) * L;
  const double2* Gr = Gs + (size_t)s * L * rpad;
  int jr[TB];  // right-hand-side columns clamped into the padded width (see k_scatter_mm)
#pragma unroll
  for (int t = 0; t < TB; ++t) jr[t] = min(rb0 + 16 * t + i, rpad - 1);
  // (four real products per k-step here: Gauss's three, with a third accumulator per block, made
  // this launch slower, 19.4 -> 21.0 ms for 64 sources at 2048^2)
  V4 cr[TB], ci[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    cr[t] = V4{0, 0, 0, 0};
    ci[t] = V4{0, 0, 0, 0};
  }
  for (int c = 0; c < L; c += 4 * KB) {
    double2 av[KB], bv[KB][TB];
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int col = c + 4 * b + k;
      const int cc = col < L ? col : L - 1;
      av[b] = Wr[cc];
#pragma unroll
      for (int t = 0; t < TB; ++t) bv[b][t] = Gr[(size_t)cc * rpad + jr[t]];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const double ok = (c + 4 * b + k < L) ? 1.0 : 0.0;
      const double ar = av[b].x * ok, ai = av[b].y * ok;
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        cr[t] = A::mma(ar, bv[b][t].x, cr[t]);
        ci[t] = A::mma(ar, bv[b][t].y, ci[t]);
        cr[t] = A::mma(-ai, bv[b][t].y, cr[t]);
        ci[t] = A::mma(ai, bv[b][t].x, ci[t]);
      }
    }
  }
  const int ndom = g.n1 * g.n2;
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
#pragma unroll
  for (int t = 0; t < TB; ++t)
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) {
      const int p = p0 + A::row_of(lane, reg), r = rb0 + 16 * t + (lane & 15);
      if (p >= g.nloc || r >= nrhs) continue;
      const int ly = p / g.snx, lx = p - ly * g.snx;
      double2* up = u + (size_t)r * g.nx * g.ny + (size_t)(y0 + ly) * g.nx + x0 + lx;
      double2 b = nz[(size_t)r * ndom + s] ? *up : mk(0.0, 0.0);
      b.x += cr[t][reg];
      b.y += ci[t][reg];
      *up = b;
    }
}

}  // namespace

hipError_t launch_recon_mm(const Geom& g, const IfCoef* coef, const FaceTab* ft, const double2* W, const double2* gin,
                           const int32_t* nz, int nrhs, double2* Gbuf, double2* u, hipStream_t st) {
  const int rpad = (nrhs + 15) / 16 * 16;
  const int ndom = g.n1 * g.n2;
  const dim3 gg((local_if_len(g) + kGP - 1) / kGP, ndom, (rpad + 63) / 64);
  hipLaunchKernelGGL(k_gather_incoming<double2>, gg, dim3(256), 0, st, g, (const int32_t*)nullptr, ft, gin, nrhs,
                     rpad, Gbuf, coef);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((g.nloc + 63) / 64, ndom, (nrhs + 16 * TB - 1) / (16 * TB));
  hipLaunchKernelGGL((k_recon_mm<4>), grid, dim3(256), 0, st, g, W, Gbuf, nrhs, rpad, nz, u);
  return hipGetLastError();
}

template <typename GT>
hipError_t launch_gather_incoming(const Geom& g, const int32_t* subs, int nsub, const FaceTab* ft, const double2* gin,
                                  int nrhs, int rpad, GT* G, hipStream_t st) {
  if (nsub == 0) return hipSuccess;
  const dim3 gg((local_if_len(g) + kGP - 1) / kGP, nsub, (rpad + 63) / 64);
  hipLaunchKernelGGL(k_gather_incoming<GT>, gg, dim3(256), 0, st, g, subs, ft, gin, nrhs, rpad, G,
                     (const IfCoef*)nullptr);
  return hipGetLastError();
}
template hipError_t launch_gather_incoming<double2>(const Geom&, const int32_t*, int, const FaceTab*, const double2*,
                                                    int, int, double2*, hipStream_t);

template <typename GT>
hipError_t launch_pregather(const int64_t* dst, const int32_t* pos, int njobs, const double2* gin, int nif, int nrhs,
                            int rpad, GT* tiles, hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  const dim3 gg((njobs + kGP - 1) / kGP, (rpad + 63) / 64);
  hipLaunchKernelGGL(k_pregather<GT>, gg, dim3(256), 0, st, dst, pos, njobs, gin, nif, nrhs, rpad, tiles);
  return hipGetLastError();
}
template hipError_t launch_pregather<double2>(const int64_t*, const int32_t*, int, const double2*, int, int, int,
                                              double2*, hipStream_t);
template hipError_t launch_pregather<float2>(const int64_t*, const int32_t*, int, const double2*, int, int, int,
                                             float2*, hipStream_t);
template hipError_t launch_gather_incoming<float2>(const Geom&, const int32_t*, int, const FaceTab*, const double2*,
                                                   int, int, float2*, hipStream_t);

template <typename C>
hipError_t launch_scatter_mm(const Geom& g, const int32_t* subs, int nsub, int mask, const FaceTab* ft, const C* T,
                             const double2* gin, const C* G, int nrhs, int rpad, const SolveIO& io, hipStream_t st,
                             int variant) {
  if (nsub == 0 || nrhs < 1) return hipSuccess;
  int rows = 0;
  for (int f = 0; f < 4; ++f)
    if ((mask >> f) & 1) rows += face_len(g, f);
  const dim3 grid((rows + 15) / 16, nsub, (nrhs + 16 * TB - 1) / (16 * TB));
  typedef typename std::conditional<sizeof(C) == 16, double, float>::type M;
  auto go = [&](auto kern, auto src, int ns, int kw = KW) {
    hipLaunchKernelGGL(kern, grid, dim3(64 * kw * ns), 0, st, g, subs, mask, ft, T, src, nrhs, rpad, io);
  };
  switch (variant) {
    case 0: go(k_scatter_mm<C, M, 2, false, 1>, G, 1); break;
    case 1: go(k_scatter_mm<C, M, 4, false, 1>, G, 1); break;
    case 2: go(k_scatter_mm<C, M, 8, false, 1>, G, 1); break;
    case 3: go(k_scatter_mm<C, M, 2, true, 1>, gin, 1); break;
    case 4: go(k_scatter_mm<C, M, 4, true, 1>, gin, 1); break;
    case 5: go(k_scatter_mm<C, M, 8, true, 1>, gin, 1); break;
    case 6: go(k_scatter_mm<C, M, 2, false, 2>, G, 2); break;
    case 7: go(k_scatter_mm<C, M, 4, false, 2>, G, 2); break;
    case 8: go(k_scatter_mm<C, M, 8, false, 2>, G, 2); break;
    case 9: go(k_scatter_mm<C, M, 2, true, 2>, gin, 2); break;
    case 10: go(k_scatter_mm<C, M, 4, true, 2>, gin, 2); break;
    case 11: go(k_scatter_mm<C, M, 8, true, 2>, gin, 2); break;
    case 12: go(k_scatter_mm<C, M, 1, false, 2, 4, true>, G, 2); break;
    case 13: go(k_scatter_mm<C, M, 1, false, 2, 8, true>, G, 2); break;
    case 14: go(k_scatter_mm<C, M, 1, true, 2, 4, true>, gin, 2); break;
    case 15: go(k_scatter_mm<C, M, 1, true, 2, 8, true>, gin, 2); break;
    case 16: go(k_scatter_mm<C, M, 4, false, 2, 0, true>, G, 2); break;
    case 17: go(k_scatter_mm<C, M, 2, true, 2, 0, true>, gin, 2); break;
    case 18: go(k_scatter_mm<C, M, 2, false, 1, 0, false, 8>, G, 1, 8); break;
    case 19: go(k_scatter_mm<C, M, 4, false, 1, 0, false, 8>, G, 1, 8); break;
    case 20: go(k_scatter_mm<C, M, 2, true, 1, 0, false, 8>, gin, 1, 8); break;
    case 21: go(k_scatter_mm<C, M, 4, true, 1, 0, false, 8>, gin, 1, 8); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_scatter_mm<double2>(const Geom&, const int32_t*, int, int, const FaceTab*, const double2*,
                                               const double2*, const double2*, int, int, const SolveIO&, hipStream_t,
                                               int);
template hipError_t launch_scatter_mm<float2>(const Geom&, const int32_t*, int, int, const FaceTab*, const float2*,
                                              const double2*, const float2*, int, int, const SolveIO&, hipStream_t,
                                              int);
