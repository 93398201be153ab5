// Batched single-right-hand-side triangular solves with the repacked band LU factors.
//
// Each workgroup performs one local solve u = A_s^{-1} rhs (the unit of work of every
// interface operator, paper Sec. 4).  The forward solve keeps a window of
// wf = nb + kl rows of the right-hand side in LDS; per column block it gathers the
// window through the block's interchange permutation and applies the
// (nb + kl) x nb matrix Mf: the first nb rows are final, the remaining kl rows
// slide down and nb fresh rows enter.  The backward solve walks the blocks from
// the last one with a window of kv + nb rows (kv = solve_kvb: kl + ku, the bandwidth of U, or ku
// when no row was interchanged).
// Loads of Mf / Mb are coalesced along the window rows (column-major per block).
//
// The right-hand side is never materialised: the forward kernel builds it on the
// fly from the source field and the incoming Robin data g injected on the edge
// rows (g / (beta- h^2)).  The backward kernel writes the outgoing traces
// -rho g - sigma u of the edge rows as soon as they are final (Sec. 4, the local
// scattering operator), to the blocks m(j, i) of the receiving neighbours.
#include "hbj_internal.h"

namespace {

struct RhsCtx {
  const Geom& g;
  const Entry& e;
  const FaceTab& F;
  const IfCoef* coef;
  const SolveIO& io;
  int slot;
  int x0, y0;
  const double2* gin;
  __device__ RhsCtx(const Geom& g_, const Entry& e_, const FaceTab& F_, const IfCoef* c_, const SolveIO& io_,
                    int slot_)
      : g(g_), e(e_), F(F_), coef(c_), io(io_), slot(slot_) {
    x0 = (e.s % g.n1) * g.snx;
    y0 = (e.s / g.n1) * g.sny;
    gin = e.src ? io.g_b : io.g_a;
    if (gin) gin += (size_t)e.rhs * g.nif;
  }
  __device__ double2 operator()(int l) const {
    if (l >= g.nloc) return mk(0.0, 0.0);
    if (io.rhs64) return io.rhs64[(size_t)slot * g.nloc + l];
    if (io.unit) {  // unit Robin datum at local interface position e.rhs
      int f, ee;
      local_if_face(g, e.rhs, &f, &ee);
      return (l == face_node(g, f, ee) && F.in_off[f] >= 0) ? coef[F.in_off[f] + ee].inj : mk(0.0, 0.0);
    }
    const int ly = l / g.snx, lx = l - ly * g.snx;
    double2 v = mk(0.0, 0.0);
    if (io.f) v = io.f[(size_t)e.rhs * g.nx * g.ny + (size_t)(y0 + ly) * g.nx + x0 + lx];
    if (gin) {
      if (lx == 0 && F.in_off[FACE_W] >= 0) { const int q = F.in_off[FACE_W] + ly; cfma(v, coef[q].inj, gin[q]); }
      if (lx == g.snx - 1 && F.in_off[FACE_E] >= 0) { const int q = F.in_off[FACE_E] + ly; cfma(v, coef[q].inj, gin[q]); }
      if (ly == 0 && F.in_off[FACE_S] >= 0) { const int q = F.in_off[FACE_S] + lx; cfma(v, coef[q].inj, gin[q]); }
      if (ly == g.sny - 1 && F.in_off[FACE_N] >= 0) { const int q = F.in_off[FACE_N] + lx; cfma(v, coef[q].inj, gin[q]); }
    }
    return v;
  }
};

template <typename C>
__device__ inline C czero() { C z; z.x = 0; z.y = 0; return z; }

// Field outputs of the final value x of local row l.
__device__ inline void emit_field(const Geom& g, const Entry& e, const SolveIO& io, int slot, int l, double2 x) {
  if (l >= g.nloc) return;
  if (io.x64) io.x64[(size_t)slot * g.nloc + l] = x;
  if (io.u) {
    const int ly = l / g.snx, lx = l - ly * g.snx;
    const int x0 = (e.s % g.n1) * g.snx, y0 = (e.s / g.n1) * g.sny;
    io.u[(size_t)e.rhs * g.nx * g.ny + (size_t)(y0 + ly) * g.nx + x0 + lx] = x;
  }
}

// Outgoing traces -rho g - sigma x of every face of the subdomain that contains local row l.
__device__ inline void emit_traces(const Geom& g, const Entry& e, const FaceTab& F, const IfCoef* coef,
                                   const SolveIO& io, const double2* gin, int l, double2 x) {
  const int ly = l / g.snx, lx = l - ly * g.snx;
  const bool on[4] = {lx == 0, lx == g.snx - 1, ly == 0, ly == g.sny - 1};
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if (!on[f] || !((e.mask >> f) & 1) || F.out_off[f] < 0) continue;
    const int ee = (f < 2) ? ly : lx;
    const int qi = F.in_off[f] + ee, qo = F.out_off[f] + ee;
    const IfCoef c = coef[qi];
    double2 val = cmul(c.sigma, x);
    if (io.tr_reflect && gin) cfma(val, c.rho, gin[qi]);
    val = mk(-val.x, -val.y);
    const size_t o = (size_t)e.rhs * g.nif + qo;
    double2 base = io.tr_base ? io.tr_base[o] : mk(0.0, 0.0);
    base.x += io.tr_sign * val.x;
    base.y += io.tr_sign * val.y;
    io.tr_dst[o] = base;
  }
}

__device__ inline void emit(const Geom& g, const Entry& e, const FaceTab& F, const IfCoef* coef, const SolveIO& io,
                            const double2* gin, int slot, int l, double2 x) {
  if (l >= g.nloc) return;
  emit_field(g, e, io, slot, l, x);
  if (io.tr_dst) emit_traces(g, e, F, coef, io, gin, l, x);
}

// q-th edge row of a subdomain: south row, north row, then the west and east columns
// without their corners (2 snx + 2 (sny - 2) rows in all).
__device__ inline int edge_row(const Geom& g, int q) {
  if (q < g.snx) return q;
  q -= g.snx;
  if (q < g.snx) return (g.sny - 1) * g.snx + q;
  q -= g.snx;
  if (q < g.sny - 2) return (1 + q) * g.snx;
  q -= g.sny - 2;
  return (1 + q) * g.snx + g.snx - 1;
}

// Cross-lane exchange inside a quad of lanes (DPP quad_perm: no LDS round trip).
// CTRL 0xB1 swaps lanes 0<->1 and 2<->3; 0x4E swaps the pairs (lanes 0,1 <-> 2,3).
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ inline float dpp_d(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL, typename C>
__device__ inline C dpp_c(C v) {
  v.x = dpp_d<CTRL>(v.x);
  v.y = dpp_d<CTRL>(v.y);
  return v;
}

// sum over the CG adjacent lanes (CG = 1, 2 or 4, aligned in a quad) that share one window row
template <int CG, typename C>
__device__ inline C row_reduce(C acc) {
  static_assert(CG == 1 || CG == 2 || CG == 4, "column groups must fit a quad of lanes");
  if (CG >= 2) acc = cadd(acc, dpp_c<0xB1>(acc));
  if (CG >= 4) acc = cadd(acc, dpp_c<0x4E>(acc));
  return acc;
}

// Forward solve y = T_{nblk-1} ... T_0 rhs.  Lane (r, cg) owns window row r and the
// columns [cg*NC, cg*NC + NC) of every block matrix; the matrices of the next D blocks and
// the right-hand-side rows entering the window are prefetched into registers, so a block's
// critical path is LDS reads, FMAs, a cross-lane sum and one barrier.  Prefetch loads are
// issued unconditionally (indices clamped into range) so that the wait before a block's
// FMAs only covers that block's own loads.
template <typename R, int NB, int CG, int D>
__global__ __launch_bounds__(576) void k_fwd(Geom g, SolveLayout L, const Entry* ent, const FaceTab* ft,
                                             const IfCoef* coef, const typename Cplx<R>::T* __restrict__ MF,
                                             const int16_t* __restrict__ PF, const int32_t* __restrict__ PFL,
                                             SolveIO io, typename Cplx<R>::T* __restrict__ ybuf) {
  typedef typename Cplx<R>::T C;
  constexpr int NC = NB / CG;
  extern __shared__ unsigned char smem_raw[];
  const int wf = L.wf, kl = g.kl, nt = blockDim.x, tid = threadIdx.x, nblk = L.nblk;
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + wf;
  int* ident = reinterpret_cast<int*>(bufB + wf);
  const Entry e = ent[blockIdx.x];
  if (io.nz && !io.nz[(size_t)e.rhs * g.n1 * g.n2 + e.s]) return;  // zero right-hand side: x = 0
  const FaceTab F = ft[e.s];
  const RhsCtx rhs(g, e, F, coef, io, blockIdx.x);
  const int ylen = nblk * NB;
  C* y = ybuf + (size_t)blockIdx.x * ylen;
  const C* M = MF + (size_t)e.s * L.mf_per_sub;
  const int16_t* P = PF + (size_t)e.s * L.pf_per_sub;
  const int32_t* PI = PFL + (size_t)e.s * nblk;
  const int cg = tid % CG, r = tid / CG;
  const bool act = r < wf;
  const size_t bstride = (size_t)NB * wf;
  const int kstride = wf * CG, toff = act ? r * CG + cg : 0;
  const int frow = min(tid, NB - 1);

  for (int l = tid; l < ylen; l += nt) y[l] = to_c<C>(rhs(l));
  for (int b = tid; b < nblk; b += nt) ident[b] = PI[b];
  __syncthreads();
  for (int q = tid; q < wf; q += nt) bufA[q] = (q < ylen) ? y[q] : czero<C>();
  // ring of D blocks: matrix slices and the window rows entering at the end of the block,
  // loaded together so that one in-order wait covers exactly one block
  C mr[D][NC];
  C fr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const C* Mb = M + (size_t)min(d, nblk - 1) * bstride + toff;
#pragma unroll
    for (int k = 0; k < NC; ++k) mr[d][k] = Mb[k * kstride];
    fr[d] = y[min((d + 1) * NB + kl + frow, ylen - 1)];
  }
  __syncthreads();

  auto step = [&](int b, C(&m)[NC], C& f) {
    if (!ident[b]) {  // row interchanges inside this block: gather the window first
      const int16_t* Pb = P + (size_t)b * wf;
      for (int q = tid; q < wf; q += nt) bufB[q] = bufA[Pb[q]];
      __syncthreads();
      C* t = bufA;
      bufA = bufB;
      bufB = t;
    }
    // the rows entering the next window go in first, so the register is free for the
    // next prefetch (no copy of an in-flight register at the loop back-edge)
    if (tid < NB) bufB[kl + tid] = ((b + 1) * NB + kl + tid < ylen) ? f : czero<C>();
    C acc = czero<C>();
#pragma unroll
    for (int k = 0; k < NC; ++k) cfma(acc, m[k], bufA[cg * NC + k]);
    acc = row_reduce<CG>(acc);
    {
      const C* Mb = M + (size_t)min(b + D, nblk - 1) * bstride + toff;
#pragma unroll
      for (int k = 0; k < NC; ++k) m[k] = Mb[k * kstride];
      f = y[min((b + D + 1) * NB + kl + frow, ylen - 1)];
    }
    if (act && cg == 0) {
      if (r < NB) y[b * NB + r] = acc;
      else bufB[r - NB] = cadd(acc, bufA[r]);
    }
    __syncthreads();
    C* t = bufA;
    bufA = bufB;
    bufB = t;
  };
  const int nmain = (nblk / D) * D;
  for (int b0 = 0; b0 < nmain; b0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) step(b0 + d, mr[d], fr[d]);
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (nmain + d < nblk) step(nmain + d, mr[d], fr[d]);
}

// Backward solve x = U^{-1} y, blocks from the last one; the window holds the block rows
// and the kl + ku rows above them that still await this block's contribution.
template <typename R, int NB, int CG, int D>
__global__ __launch_bounds__(576) void k_bwd(Geom g, SolveLayout L, const Entry* ent, const FaceTab* ft,
                                             const IfCoef* coef, const typename Cplx<R>::T* __restrict__ MB,
                                             SolveIO io, typename Cplx<R>::T* __restrict__ ybuf) {
  typedef typename Cplx<R>::T C;
  constexpr int NC = NB / CG;
  extern __shared__ unsigned char smem_raw[];
  const int wb = L.wb, kv = solve_kvb(L), nt = blockDim.x, tid = threadIdx.x, nblk = L.nblk;
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + wb;
  const Entry e = ent[blockIdx.x];
  const FaceTab F = ft[e.s];
  const int ylen = nblk * NB;
  C* y = ybuf + (size_t)blockIdx.x * ylen;
  const C* M = MB + (size_t)e.s * L.mb_per_sub;
  const double2* gin = e.src ? io.g_b : io.g_a;
  if (gin) gin += (size_t)e.rhs * g.nif;
  if (io.nz && !io.nz[(size_t)e.rhs * g.n1 * g.n2 + e.s]) {  // zero right-hand side: x = 0
    if (io.nz_skip_out) return;
    if (io.u || io.x64)
      for (int l = threadIdx.x; l < g.nloc; l += blockDim.x) emit_field(g, e, io, blockIdx.x, l, mk(0.0, 0.0));
    if (io.tr_dst) {
      const int nedge = 2 * g.snx + 2 * (g.sny - 2);
      for (int q = threadIdx.x; q < nedge; q += blockDim.x)
        emit_traces(g, e, F, coef, io, gin, edge_row(g, q), mk(0.0, 0.0));
    }
    return;
  }
  const int cg = tid % CG, r = tid / CG;
  const bool act = r < wb;
  const size_t bstride = (size_t)NB * wb;
  const int kstride = wb * CG, toff = act ? r * CG + cg : 0;
  const int frow = min(tid, NB - 1);

  {
    const int j0 = (nblk - 1) * NB;
    for (int q = tid; q < wb; q += nt) {
      const int row = j0 - kv + q;
      bufA[q] = (row >= 0) ? y[row] : czero<C>();
    }
  }
  C mr[D][NC];
  C fr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const C* Mb = M + (size_t)max(nblk - 1 - d, 0) * bstride + toff;
#pragma unroll
    for (int k = 0; k < NC; ++k) mr[d][k] = Mb[k * kstride];
    fr[d] = y[max((nblk - 2 - d) * NB - kv + frow, 0)];
  }
  __syncthreads();

  auto step = [&](int b, C(&m)[NC], C& f) {
    if (tid < NB) bufB[tid] = ((b - 1) * NB - kv + tid >= 0) ? f : czero<C>();
    C acc = czero<C>();
#pragma unroll
    for (int k = 0; k < NC; ++k) cfma(acc, m[k], bufA[kv + cg * NC + k]);
    acc = row_reduce<CG>(acc);
    {
      const C* Mb = M + (size_t)max(b - D, 0) * bstride + toff;
#pragma unroll
      for (int k = 0; k < NC; ++k) m[k] = Mb[k * kstride];
      f = y[max((b - D - 1) * NB - kv + frow, 0)];
    }
    if (act && cg == 0) {
      if (r >= kv) y[b * NB + r - kv] = acc;
      else bufB[r + NB] = cadd(acc, bufA[r]);
    }
    __syncthreads();
    C* t = bufA;
    bufA = bufB;
    bufB = t;
  };
  const int nmain = (nblk / D) * D;
  for (int i0 = 0; i0 < nmain; i0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) step(nblk - 1 - (i0 + d), mr[d], fr[d]);
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (nmain + d < nblk) step(nblk - 1 - (nmain + d), mr[d], fr[d]);
  // the solution is final: write the requested outputs
  if (io.u || io.x64) {
    for (int l = tid; l < g.nloc; l += nt) emit_field(g, e, io, blockIdx.x, l, to_d(y[l]));
  }
  if (io.tr_dst) {
    const int nedge = 2 * g.snx + 2 * (g.sny - 2);
    for (int q = tid; q < nedge; q += nt) {
      const int l = edge_row(g, q);
      emit_traces(g, e, F, coef, io, gin, l, to_d(y[l]));
    }
  }
}

// nz[rhs][s] = 1 if the source restricted to subdomain s is not identically zero.  Each thread
// issues the loads of kFlagU positions (clamped into the subdomain: a repeated position does not
// change the result) before it tests any, so a 128^2 subdomain costs one round of loads.
constexpr int kFlagThreads = 1024, kFlagU = 16;
__global__ __launch_bounds__(kFlagThreads) void k_source_flags(Geom g, const double2* f, int32_t* nz) {
  const int s = blockIdx.x, rhs = blockIdx.y;
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
  const double2* fr = f + (size_t)rhs * g.nx * g.ny;
  int any = 0;
  for (int l0 = 0; l0 < g.nloc; l0 += kFlagU * kFlagThreads) {
    double2 v[kFlagU];
#pragma unroll
    for (int u = 0; u < kFlagU; ++u) {
      const int l = min(l0 + (int)threadIdx.x + u * kFlagThreads, g.nloc - 1);
      const int ly = l / g.snx, lx = l - ly * g.snx;
      v[u] = fr[(size_t)(y0 + ly) * g.nx + x0 + lx];
    }
#pragma unroll
    for (int u = 0; u < kFlagU; ++u) any |= (v[u].x != 0.0) | (v[u].y != 0.0);
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) nz[(size_t)rhs * g.n1 * g.n2 + s] = any;
}

// explicit complex128 right-hand sides (source + injected Robin data) of a batch
__global__ void k_build_rhs(Geom g, const Entry* ent, const FaceTab* ft, const IfCoef* coef, SolveIO io,
                            double2* rhs64) {
  const int slot = blockIdx.y;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= g.nloc) return;
  const Entry e = ent[slot];
  const FaceTab F = ft[e.s];
  const RhsCtx rhs(g, e, F, coef, io, slot);
  rhs64[(size_t)slot * g.nloc + l] = rhs(l);
}

// outgoing traces of complex128 local solutions x64 [entry][nloc]
// Outgoing traces of every masked face from whole local fields x64[slot] (after the solves):
// -sum_d R[e][e+d] g - sum_d Sigma[e][e+d] x along the face (the band rows of the transmission
// condition; first order: -rho g - sigma x at the node), then the field outputs of io.
__global__ void k_emit_traces(Geom g, const Entry* ent, const FaceTab* ft, const IfBand* band, SolveIO io,
                              const double2* x64) {
  const int slot = blockIdx.y;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= g.nloc) return;
  const int ly = l / g.snx, lx = l - ly * g.snx;
  if (!(lx == 0 || lx == g.snx - 1 || ly == 0 || ly == g.sny - 1)) return;
  const Entry e = ent[slot];
  const FaceTab F = ft[e.s];
  const double2* gin = e.src ? io.g_b : io.g_a;
  if (gin) gin += (size_t)e.rhs * g.nif;
  const double2* xs = x64 + (size_t)slot * g.nloc;
  emit_field(g, e, io, slot, l, xs[l]);
  if (!io.tr_dst) return;
  const bool on[4] = {lx == 0, lx == g.snx - 1, ly == 0, ly == g.sny - 1};
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if (!on[f] || !((e.mask >> f) & 1) || F.out_off[f] < 0) continue;
    const int ee = (f < 2) ? ly : lx;
    const int len = f < 2 ? g.sny : g.snx;
    const int qi = F.in_off[f] + ee, qo = F.out_off[f] + ee;
    const IfBand B = band[qi];
    double2 val = mk(0.0, 0.0);
    for (int d = 0; d < 5; ++d) {
      const int xx = ee + d - 2;
      if (xx >= 0 && xx < len) cfma(val, B.sg[d], xs[face_node(g, f, xx)]);
    }
    if (io.tr_reflect && gin)
      for (int d = 0; d < 3; ++d) {
        const int xx = ee + d - 1;
        if (xx >= 0 && xx < len) cfma(val, B.r[d], gin[F.in_off[f] + xx]);
      }
    val = mk(-val.x, -val.y);
    const size_t o = (size_t)e.rhs * g.nif + qo;
    double2 base = io.tr_base ? io.tr_base[o] : mk(0.0, 0.0);
    base.x += io.tr_sign * val.x;
    base.y += io.tr_sign * val.y;
    io.tr_dst[o] = base;
  }
}

// x64 += dx for complex64 corrections held in the solve buffer [entry][nblk * nb]
__global__ void k_axpy_c64(double2* x64, const float2* dx, int nloc, int stride) {
  const int slot = blockIdx.y;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nloc) return;
  const float2 d = dx[(size_t)slot * stride + l];
  double2& x = x64[(size_t)slot * nloc + l];
  x.x += (double)d.x;
  x.y += (double)d.y;
}

// ---------------------------------------------------------------------------
// Many right-hand sides of one subdomain per workgroup, on MFMA.
//
// A tile is a run of up to 16 entries of a launch that share one subdomain.  For those right-hand
// sides the block recurrence of k_fwd / k_bwd becomes one complex matrix product per column
// block, acc = M_b (window rows x 16) * X_b (16 x 16 right-hand sides), X_b being the rows of the
// window that the block eliminates; each complex k-step is four real 16x16x4 MFMAs (Re += Ar Br -
// Ai Bi, Im += Ar Bi + Ai Br).  The window is padded to NT whole tiles of 16 rows (padding rows
// have zero multipliers and only carry their values) and lives in the MFMA accumulators: physical
// tile p belongs to wavefront p % 4 and the window slides by renaming (logical tile t of a block
// is a fixed physical tile shifted by the block index modulo NT), so no row ever moves between
// registers.  Per block every wavefront multiplies its tiles by X_b; the tile that becomes the
// next block's X is written to LDS, double-buffered, so one barrier per block suffices.  Blocks
// with row interchanges pass the window through LDS.  Lane l works on right-hand side l % 16; the
// loads of the next block's multipliers and of the rows entering the window are issued before the
// current block's products.

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename C, typename R>
__device__ inline C mkc(R x, R y) {
  C v;
  v.x = x;
  v.y = y;
  return v;
}

template <typename R> struct TriMma;
template <> struct TriMma<double> {
  typedef d4v V;
  static __device__ inline V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // accumulator register r of lane l holds row row_of(l, r), column l % 16
  static __device__ inline int row_of(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct TriMma<float> {
  typedef f4v V;
  static __device__ inline V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row_of(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// acc_si += A_si X for the SPW tiles of a wavefront (a[si][ks]: this lane's multipliers, row lane % 16,
// column 4 ks + lane / 16, times ok[si], 0 for rows outside the band; x: this lane's X operands),
// k-steps outermost so that consecutive MFMAs go to independent accumulators
template <typename R, int SPW>
__device__ inline void tiles_mma(const typename Cplx<R>::T (&a)[SPW][4], const R (&ok)[SPW], const R (&xr)[4],
                                 const R (&xi)[4],
                                 typename TriMma<R>::V (&wr)[SPW], typename TriMma<R>::V (&wi)[SPW]) {
  typedef TriMma<R> T;
  R nxi[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) nxi[ks] = -xi[ks];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int si = 0; si < SPW; ++si) {
      const R ar = (R)a[si][ks].x * ok[si], ai = (R)a[si][ks].y * ok[si];
      wr[si] = T::mma(ar, xr[ks], wr[si]);
      wi[si] = T::mma(ar, xi[ks], wi[si]);
      wr[si] = T::mma(ai, nxi[ks], wr[si]);
      wi[si] = T::mma(ai, xr[ks], wi[si]);
    }
}


// Per-wavefront state of the MFMA band solves: wavefront w holds the logical window tiles
// w SPW + si (si < SPW) in accumulators, so every tile keeps one role (and one set of load
// offsets and row masks) for the whole solve; the window slides by moving tiles one slot along,
// the tile that leaves a wavefront's range passing to the neighbouring wavefront through LDS.
template <typename R, int SPW>
struct MmWin {
  typedef typename TriMma<R>::V V;
  V wr[SPW], wi[SPW];
  __device__ inline void zero(int si) {
    wr[si] = V{0, 0, 0, 0};
    wi[si] = V{0, 0, 0, 0};
  }
  template <typename C>
  __device__ inline void set(int si, const C (&v)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      wr[si][r] = (R)v[r].x;
      wi[si][r] = (R)v[r].y;
    }
  }
  // tile si to LDS as [16 rows][16 right-hand sides] (this lane: rows row_of(lane, r), column lane % 16)
  template <typename C>
  __device__ inline void put(int si, C* dst, int lane) const {
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[TriMma<R>::row_of(lane, r) * 16 + (lane & 15)] = mkc<C, R>(wr[si][r], wi[si][r]);
  }
  template <typename C>
  __device__ inline void get(int si, const C* src, int lane) {
    C v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = src[TriMma<R>::row_of(lane, r) * 16 + (lane & 15)];
    set(si, v);
  }
};

// Every global load and store of the block loops is issued by every lane on every path (rows out of
// range are clamped and replaced where they are used; the final rows of a block are stored by all
// four wavefronts from LDS, lanes without a right-hand side writing to a sink), so the compiler can
// count the loads in flight exactly and waits only for the previous block's.  PIV: the subdomains may
// have row interchanges (a per-block flag and permutation; otherwise the flags are not read).
template <typename R, int SPW, bool PIV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_fwd_mm(
    Geom g, SolveLayout L, const Entry* ent, const int2* tiles, const FaceTab* ft, const IfCoef* coef,
    const typename Cplx<R>::T* __restrict__ MF, const int16_t* __restrict__ PF, const int32_t* __restrict__ PFL,
    SolveIO io, typename Cplx<R>::T* __restrict__ ybuf, typename Cplx<R>::T* __restrict__ sink) {
  typedef typename Cplx<R>::T C;
  typedef TriMma<R> T;
  constexpr int NT = 4 * SPW;  // window tiles; rows past wf have zero multipliers
  extern __shared__ unsigned char smem_raw[];
  const int nblk = L.nblk, wf = L.wf, ylen = nblk * 16;
  C* xsh = reinterpret_cast<C*>(smem_raw);                               // [2][16 rows][16]: X of a block
  int* ident = reinterpret_cast<int*>(xsh + 512);                        // [nblk] (PIV)
  C* wsh = reinterpret_cast<C*>(ident + (PIV ? ((nblk + 3) & ~3) : 0));  // [NT * 16][16] interchanges, or:
  C* bsh = wsh;                                                          // [2][3][16][16] tiles passed on
  C* ysh = wsh + 6 * 256;                                                // [2][16][16] final rows
  const int tix = xcd_tile(blockIdx.x, gridDim.x);
  const int2 tl = make_int2(__builtin_amdgcn_readfirstlane(tiles[tix].x),
                            __builtin_amdgcn_readfirstlane(tiles[tix].y));  // first entry, count (1..16)
  const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool mine = j < tl.y;  // lanes past the count work on a copy of the first entry, unstored
  const int s = __builtin_amdgcn_readfirstlane(ent[tl.x].s);
  const FaceTab F = ft[s];
  const C* M = MF + (size_t)s * L.mf_per_sub;
  const int16_t* P = PF + (size_t)s * L.pf_per_sub;
  C* y = ybuf + (size_t)tl.x * ylen;                      // the tile's first solve buffer (uniform)
  const unsigned yl = (unsigned)((mine ? j : 0) * ylen);  // this lane's, relative to it
  C* yout = mine ? ybuf + (size_t)(tl.x + j) * ylen : sink;  // where this lane's final rows go
  if (PIV)
    for (int b = threadIdx.x; b < nblk; b += 256) ident[b] = PFL[(size_t)s * nblk + b];
  {  // the right-hand sides into the solve buffers (the window reads them ahead of the solution)
    const int jj = threadIdx.x & 15;
    if (jj < tl.y) {
      const Entry ej = ent[tl.x + jj];
      const bool zj = io.nz && !io.nz[(size_t)ej.rhs * g.n1 * g.n2 + ej.s];
      const RhsCtx rj(g, ej, F, coef, io, tl.x + jj);
      C* yj = ybuf + (size_t)(tl.x + jj) * ylen;
      for (int l = threadIdx.x >> 4; l < ylen; l += 16) yj[l] = zj ? czero<C>() : to_c<C>(rj(l));
    }
  }
  __syncthreads();

  // rows row0 + [0, 16) of the right-hand sides (row0 a multiple of 16): always loaded (clamped into
  // the buffer), so that the number of loads in flight is the same on every path; rows past the end
  // are replaced by zeros where they enter the window
  auto fresh = [&](int row0, C(&v)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = y[yl + (unsigned)min(row0 + T::row_of(lane, r), ylen - 1)];
  };
  // multipliers: entry (row r, column 4 ks + q) of a block lies at (q wf + r) cg + kofs[ks] in the
  // tiled layout; the row of tile si is 16 (w SPW + si) + j (clamped, masked by ok)
  const int cg = L.cgf, nc = 16 / cg;
  int kofs[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) kofs[ks] = ((4 * ks) % nc) * wf * cg + (4 * ks) / nc;
  unsigned lo[SPW];
  R ok[SPW];
#pragma unroll
  for (int si = 0; si < SPW; ++si) {
    const int row = 16 * (w * SPW + si) + j;
    lo[si] = (unsigned)((q * wf + min(row, wf - 1)) * cg) * (unsigned)sizeof(C);
    ok[si] = row < wf ? (R)1 : (R)0;
  }
  auto load_a = [&](int b, C(&a)[SPW][4]) {
    const C* Mb = M + (size_t)b * 16 * wf;
#pragma unroll
    for (int si = 0; si < SPW; ++si)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        a[si][ks] = *reinterpret_cast<const C*>(reinterpret_cast<const char*>(Mb + kofs[ks]) + lo[si]);
  };

  MmWin<R, SPW> W;
  C a0[SPW][4], a1[SPW][4];
  C f0[4], f1[4];
#pragma unroll
  for (int si = 0; si < SPW; ++si) {
    C v[4];
    fresh(16 * (w * SPW + si), v);
    if (16 * (w * SPW + si) < ylen) W.set(si, v);
    else W.zero(si);
  }
  load_a(0, a0);
  fresh(NT * 16, f0);  // used by wavefront 3
  if (w == 0) {  // X of block 0 is logical tile 0; that tile then starts from zero
    W.put(0, xsh, lane);
    W.zero(0);
  }
  __syncthreads();

  auto block = [&](int b, C(&acur)[SPW][4], C(&anxt)[SPW][4], C(&fr)[4], C(&frn)[4]) {
    const int par = b & 1;
    load_a(min(b + 1, nblk - 1), anxt);
    fresh((b + 1 + NT) * 16, frn);  // used by wavefront 3; loaded by all so that the load count is static
    R xr[4], xi[4];
    if (PIV && !__builtin_amdgcn_readfirstlane(ident[b])) {  // row interchanges: gather the window through LDS
      __syncthreads();  // the scratch also holds the tiles passed on at the end of the last block
#pragma unroll
      for (int si = 0; si < SPW; ++si) {
        C* dst = wsh + (w * SPW + si) * 256;
        if (w == 0 && si == 0) {  // logical tile 0 is X (its accumulator was cleared)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = T::row_of(lane, r) * 16 + j;
            dst[o] = xsh[par * 256 + o];
          }
        } else {
          W.put(si, dst, lane);
        }
      }
      __syncthreads();
      const int16_t* Pb = P + (size_t)b * wf;
#pragma unroll
      for (int si = 0; si < SPW; ++si) {
        C v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (w * SPW + si) + T::row_of(lane, r);
          v[r] = wsh[(row < wf ? (int)Pb[row] : row) * 16 + j];
        }
        W.set(si, v);
      }
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const C v = wsh[(int)Pb[4 * ks + q] * 16 + j];
        xr[ks] = (R)v.x;
        xi[ks] = (R)v.y;
      }
      if (w == 0) W.zero(0);
      __syncthreads();
    } else {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const C v = xsh[par * 256 + (4 * ks + q) * 16 + j];
        xr[ks] = (R)v.x;
        xi[ks] = (R)v.y;
      }
    }
    tiles_mma<R, SPW>(acur, ok, xr, xi, W.wr, W.wi);
    // logical tile 0 holds the block's final rows; tile 1 is the next block's X; the window moves
    // down one tile: every tile goes one slot lower, slot 0 of wavefronts 1-3 to the wavefront below
    if (w == 0) W.put(0, ysh + par * 256, lane);
    else W.put(0, bsh + (par * 3 + w - 1) * 256, lane);
    if (SPW >= 2) {
      if (w == 0) W.put(1, xsh + (par ^ 1) * 256, lane);
    } else {
      if (w == 1) W.put(0, xsh + (par ^ 1) * 256, lane);
    }
#pragma unroll
    for (int si = 0; si + 1 < SPW; ++si) {
      W.wr[si] = W.wr[si + 1];
      W.wi[si] = W.wi[si + 1];
    }
    if (SPW >= 2 && w == 0) W.zero(0);  // the next block's X: its tile starts from zero
    __syncthreads();
    yout[b * 16 + 4 * w + q] = ysh[par * 256 + (4 * w + q) * 16 + j];  // rows 4 w + [0, 4) of the final rows
    if (w == 3) {  // rows entering the window
      if ((b + NT) * 16 < ylen) W.set(SPW - 1, fr);
      else W.zero(SPW - 1);
    } else if (SPW == 1 && w == 0) {
      W.zero(0);
    } else {
      W.get(SPW - 1, bsh + (par * 3 + w) * 256, lane);
    }
  };
  int b = 0;
  for (; b + 1 < nblk; b += 2) {  // two blocks per trip: the register sets swap roles without copies
    block(b, a0, a1, f0, f1);
    block(b + 1, a1, a0, f1, f0);
  }
  if (b < nblk) block(b, a0, a1, f0, f1);
}

template <typename R, int SPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_bwd_mm(
    Geom g, SolveLayout L, const Entry* ent, const int2* tiles, const FaceTab* ft, const IfCoef* coef,
    const typename Cplx<R>::T* __restrict__ MB, SolveIO io, typename Cplx<R>::T* __restrict__ ybuf,
    typename Cplx<R>::T* __restrict__ sink) {
  typedef typename Cplx<R>::T C;
  typedef TriMma<R> T;
  constexpr int NT = 4 * SPW;  // window tiles; rows above the band have zero multipliers
  extern __shared__ unsigned char smem_raw[];
  const int nblk = L.nblk, wb = L.wb, pad = NT * 16 - wb, ylen = nblk * 16;
  C* xsh = reinterpret_cast<C*>(smem_raw);  // [2][16 rows][16]: X of a block
  C* bsh = xsh + 512;                       // [2][3][16][16]: tiles passed on
  C* ysh = bsh + 6 * 256;                   // [2][16][16]: final rows
  const int tix = xcd_tile(blockIdx.x, gridDim.x);
  const int2 tl = make_int2(__builtin_amdgcn_readfirstlane(tiles[tix].x), __builtin_amdgcn_readfirstlane(tiles[tix].y));
  const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool mine = j < tl.y;
  const int s = __builtin_amdgcn_readfirstlane(ent[tl.x].s);
  const C* M = MB + (size_t)s * L.mb_per_sub;
  C* y = ybuf + (size_t)tl.x * ylen;                      // the tile's first solve buffer (uniform)
  const unsigned yl = (unsigned)((mine ? j : 0) * ylen);  // this lane's, relative to it
  C* yout = mine ? ybuf + (size_t)(tl.x + j) * ylen : sink;  // where this lane's final rows go
  // logical tile u of the step for block b holds rows b*16 - (NT - 1 - u)*16 + [0, 16), window
  // rows 16 u - pad + [0, 16) of k_bwd
  // rows row0 + [0, 16) of y (row0 a multiple of 16): always loaded (clamped to row 0 above the
  // matrix), rows above the matrix replaced by zeros where they enter the window
  auto fresh = [&](int row0, C(&v)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = y[yl + (unsigned)max(row0 + T::row_of(lane, r), 0)];
  };
  const int cg = L.cgb, nc = 16 / cg;
  int kofs[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) kofs[ks] = ((4 * ks) % nc) * wb * cg + (4 * ks) / nc;
  unsigned lo[SPW];
  R ok[SPW];
#pragma unroll
  for (int si = 0; si < SPW; ++si) {
    const int row = 16 * (w * SPW + si) + j - pad;
    lo[si] = (unsigned)((q * wb + max(row, 0)) * cg) * (unsigned)sizeof(C);
    ok[si] = row >= 0 ? (R)1 : (R)0;
  }
  auto load_a = [&](int b, C(&a)[SPW][4]) {
    const C* Mb = M + (size_t)b * 16 * wb;
#pragma unroll
    for (int si = 0; si < SPW; ++si)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        a[si][ks] = *reinterpret_cast<const C*>(reinterpret_cast<const char*>(Mb + kofs[ks]) + lo[si]);
  };

  MmWin<R, SPW> W;
  C a0[SPW][4], a1[SPW][4];
  C f0[4], f1[4];
#pragma unroll
  for (int si = 0; si < SPW; ++si) {
    C v[4];
    fresh((nblk - NT + w * SPW + si) * 16, v);
    if (nblk - NT + w * SPW + si >= 0) W.set(si, v);
    else W.zero(si);
  }
  load_a(nblk - 1, a0);
  fresh((nblk - 1 - NT) * 16, f0);  // used by wavefront 0
  if (w == 3) {  // X of the last block is logical tile NT - 1; that tile then starts from zero
    W.put(SPW - 1, xsh, lane);
    W.zero(SPW - 1);
  }
  __syncthreads();

  auto step = [&](int i, C(&acur)[SPW][4], C(&anxt)[SPW][4], C(&fr)[4], C(&frn)[4]) {
    const int b = nblk - 1 - i, par = i & 1;
    load_a(max(b - 1, 0), anxt);
    fresh((b - 1 - NT) * 16, frn);  // used by wavefront 0; loaded by all so that the load count is static
    R xr[4], xi[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const C v = xsh[par * 256 + (4 * ks + q) * 16 + j];
      xr[ks] = (R)v.x;
      xi[ks] = (R)v.y;
    }
    tiles_mma<R, SPW>(acur, ok, xr, xi, W.wr, W.wi);
    // logical tile NT - 1 holds the block's unknowns; tile NT - 2 is the next block's X; the window
    // moves up one tile: every tile goes one slot higher, the last slot of wavefronts 0-2 to the next
    if (w == 3) W.put(SPW - 1, ysh + par * 256, lane);
    else W.put(SPW - 1, bsh + (par * 3 + w) * 256, lane);
    if (SPW >= 2) {
      if (w == 3) W.put(SPW - 2, xsh + (par ^ 1) * 256, lane);
    } else {
      if (w == 2) W.put(0, xsh + (par ^ 1) * 256, lane);
    }
#pragma unroll
    for (int si = SPW - 1; si > 0; --si) {
      W.wr[si] = W.wr[si - 1];
      W.wi[si] = W.wi[si - 1];
    }
    if (SPW >= 2 && w == 3) W.zero(SPW - 1);  // the next block's X: its tile starts from zero
    __syncthreads();
    yout[b * 16 + 4 * w + q] = ysh[par * 256 + (4 * w + q) * 16 + j];  // rows 4 w + [0, 4) of the unknowns
    if (w == 0) {  // rows entering the window
      if (b - NT >= 0) W.set(0, fr);
      else W.zero(0);
    } else if (SPW == 1 && w == 3) {
      W.zero(0);
    } else {
      W.get(0, bsh + (par * 3 + w - 1) * 256, lane);
    }
  };
  int i = 0;
  for (; i + 1 < nblk; i += 2) {
    step(i, a0, a1, f0, f1);
    step(i + 1, a1, a0, f1, f0);
  }
  if (i < nblk) step(i, a0, a1, f0, f1);
  __syncthreads();
  // the solutions are final: the outputs of every entry of the tile, as k_bwd writes them
  const FaceTab F = ft[s];
  const int cnt = tl.y, nloc = g.nloc;
  if (io.u || io.x64) {
    for (int idx = threadIdx.x; idx < cnt * nloc; idx += 256) {
      const int jj = idx / nloc, l = idx - jj * nloc, sl = tl.x + jj;
      const Entry ej = ent[sl];
      if (io.nz && io.nz_skip_out && !io.nz[(size_t)ej.rhs * g.n1 * g.n2 + ej.s]) continue;
      emit_field(g, ej, io, sl, l, to_d(ybuf[(size_t)sl * ylen + l]));
    }
  }
  if (io.tr_dst) {
    const int nedge = 2 * g.snx + 2 * (g.sny - 2);
    for (int idx = threadIdx.x; idx < cnt * nedge; idx += 256) {
      const int jj = idx / nedge, qq = idx - jj * nedge, sl = tl.x + jj;
      const Entry ej = ent[sl];
      if (io.nz && io.nz_skip_out && !io.nz[(size_t)ej.rhs * g.n1 * g.n2 + ej.s]) continue;
      const double2* gin = ej.src ? io.g_b : io.g_a;
      if (gin) gin += (size_t)ej.rhs * g.nif;
      const int l = edge_row(g, qq);
      emit_traces(g, ej, F, coef, io, gin, l, to_d(ybuf[(size_t)sl * ylen + l]));
    }
  }
}

// ---------------------------------------------------------------------------
// One local solve split over several workgroups (partitioned substitution).
//
// The forward (backward) substitution is a linear recurrence over the column blocks whose state
// is the window part carried from one block to the next: kl rows in the forward solve, kv rows in
// the backward one.  The blocks of a subdomain split into np runs of bpp blocks (processing order
// o = 0 .. np-1: from the first block forward, from the last one backward).  Pass 1 runs every
// run but the last on its own workgroup, run 0 exactly (its incoming state is the right-hand
// side), the others from a zero incoming state, and stores their outgoing states (sig).  The chain
// recovers the true incoming state of every run, tt[o + 1] = sig[o] + Phi_o tt[o], with the runs'
// transfer matrices Phi_o (the outgoing state for each unit incoming state and no right-hand side,
// formed once per factorisation by k_part_phi_*).  Pass 2 reruns every run but the first from its
// true state and writes its rows.  Each pass reads every factor byte once, on np workgroups.
// Buffers: rb [entry][nblk nb] the right-hand sides (the first forward pass writes them: run o the
// rows it reads, up to kl + nb rows into run o + 1, which writes the same values, and a workgroup
// for the last run only its rows; building them inside the passes' prefetch path instead doubled
// the passes' time), yb the results, sig / tt [entry][np][ns] the states, Phi
// [subdomain][np - 2][S][S] column-major (S = kl or kv).

// Chain states not yet written hold a signalling-NaN bit pattern, which no arithmetic result has
// (operations return quiet NaNs): the chain's tasks poll their input state until no entry holds it.
constexpr unsigned long long kUnset64 = 0x7FF4A5A5A5A5A5A5ull;
constexpr unsigned kUnset32 = 0x7FA5A5A5u;
__device__ inline void set_unset(double2& v) {
  v.x = __longlong_as_double((long long)kUnset64);
  v.y = v.x;
}
__device__ inline void set_unset(float2& v) {
  v.x = __int_as_float((int)kUnset32);
  v.y = v.x;
}
__device__ inline bool is_unset(double2 v) {
  return (unsigned long long)__double_as_longlong(v.x) == kUnset64 ||
         (unsigned long long)__double_as_longlong(v.y) == kUnset64;
}
__device__ inline bool is_unset(float2 v) {
  return (unsigned)__float_as_int(v.x) == kUnset32 || (unsigned)__float_as_int(v.y) == kUnset32;
}

template <typename R, int NB, int CG, int D>
__global__ __launch_bounds__(576) void k_fwd_part(Geom g, SolveLayout L, PartLayout pl, int phase, const Entry* ent,
                                                  const FaceTab* ft, const IfCoef* coef, SolveIO io,
                                                  const typename Cplx<R>::T* __restrict__ MF,
                                                  const int16_t* __restrict__ PF, const int32_t* __restrict__ PFL,
                                                  typename Cplx<R>::T* rb, typename Cplx<R>::T* __restrict__ yb,
                                                  typename Cplx<R>::T* sig, typename Cplx<R>::T* tt) {
  typedef typename Cplx<R>::T C;
  constexpr int NC = NB / CG;
  extern __shared__ unsigned char smem_raw[];
  const int wf = L.wf, kl = g.kl, nt = blockDim.x, tid = threadIdx.x, nblk = L.nblk;
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + wf;
  int* ident = reinterpret_cast<int*>(bufB + wf);
  const int slot = blockIdx.x;
  const int o = phase == 1 ? (int)blockIdx.y : (int)blockIdx.y + 1;
  const Entry e = ent[slot];
  if (io.nz && !io.nz[(size_t)e.rhs * g.n1 * g.n2 + e.s]) return;  // zero right-hand side: x = 0
  const int b0 = o * pl.bpp, b1 = min(b0 + pl.bpp, nblk);
  const int ylen = nblk * NB;
  C* rhs = rb + (size_t)slot * ylen;
  C* y = yb + (size_t)slot * ylen;
  if (phase == 1) {  // the right-hand-side rows this run reads (the last run: its own rows only)
    const FaceTab F = ft[e.s];
    const RhsCtx rc(g, e, F, coef, io, slot);
    const int hi = o == pl.np - 1 ? ylen : min(b1 * NB + kl + NB, ylen);
    for (int l = b0 * NB + tid; l < hi; l += nt) rhs[l] = to_c<C>(rc(l));
    if (o == pl.np - 1) return;
    __syncthreads();
  }
  const bool outs = phase == 3 || o == 0;
  const C* M = MF + (size_t)e.s * L.mf_per_sub;
  const int16_t* P = PF + (size_t)e.s * L.pf_per_sub;
  const int32_t* PI = PFL + (size_t)e.s * nblk + b0;
  const int cg = tid % CG, r = tid / CG;
  const bool act = r < wf;
  const size_t bstride = (size_t)NB * wf;
  const int kstride = wf * CG, toff = act ? r * CG + cg : 0;
  const int frow = min(tid, NB - 1);

  for (int b = tid; b < b1 - b0; b += nt) ident[b] = PI[b];
  {
    const C* tin = tt + ((size_t)slot * pl.np + o) * pl.ns;
    for (int q = tid; q < wf; q += nt) {
      const int row = b0 * NB + q;
      C v = row < ylen ? rhs[row] : czero<C>();
      if (q < kl && o > 0) v = phase == 3 ? tin[q] : czero<C>();
      bufA[q] = v;
    }
  }
  C mr[D][NC];
  C fr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const C* Mb = M + (size_t)min(b0 + d, b1 - 1) * bstride + toff;
#pragma unroll
    for (int k = 0; k < NC; ++k) mr[d][k] = Mb[k * kstride];
    fr[d] = rhs[min((b0 + d + 1) * NB + kl + frow, ylen - 1)];
  }
  __syncthreads();

  auto step = [&](int b, C(&m)[NC], C& f) {
    if (!ident[b - b0]) {
      const int16_t* Pb = P + (size_t)b * wf;
      for (int q = tid; q < wf; q += nt) bufB[q] = bufA[Pb[q]];
      __syncthreads();
      C* t = bufA;
      bufA = bufB;
      bufB = t;
    }
    if (tid < NB) bufB[kl + tid] = ((b + 1) * NB + kl + tid < ylen) ? f : czero<C>();
    C acc = czero<C>();
#pragma unroll
    for (int k = 0; k < NC; ++k) cfma(acc, m[k], bufA[cg * NC + k]);
    acc = row_reduce<CG>(acc);
    {
      const C* Mb = M + (size_t)min(b + D, b1 - 1) * bstride + toff;
#pragma unroll
      for (int k = 0; k < NC; ++k) m[k] = Mb[k * kstride];
      f = rhs[min((b + D + 1) * NB + kl + frow, ylen - 1)];
    }
    if (act && cg == 0) {
      if (r < NB) {
        if (outs) y[b * NB + r] = acc;
      } else {
        bufB[r - NB] = cadd(acc, bufA[r]);
      }
    }
    __syncthreads();
    C* t = bufA;
    bufA = bufB;
    bufB = t;
  };
  const int n = b1 - b0, nmain = (n / D) * D;
  for (int i0 = 0; i0 < nmain; i0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) step(b0 + i0 + d, mr[d], fr[d]);
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (nmain + d < n) step(b0 + nmain + d, mr[d], fr[d]);
  if (phase == 1) {  // the outgoing state: window rows [0, kl) of block b1
    C* dst = o == 0 ? tt + ((size_t)slot * pl.np + 1) * pl.ns : sig + ((size_t)slot * pl.np + o) * pl.ns;
    for (int q = tid; q < kl; q += nt) dst[q] = bufA[q];
    if (o >= 1 && o + 1 <= pl.np - 1) {  // the chain's output state o + 1 starts unset
      C u;
      set_unset(u);
      for (int q = tid; q < kl; q += nt) tt[((size_t)slot * pl.np + o + 1) * pl.ns + q] = u;
    }
  }
}

template <typename R, int NB, int CG, int D>
__global__ __launch_bounds__(576) void k_bwd_part(Geom g, SolveLayout L, PartLayout pl, int phase, const Entry* ent,
                                                  const FaceTab* ft, const IfCoef* coef,
                                                  const typename Cplx<R>::T* __restrict__ MB, SolveIO io,
                                                  const typename Cplx<R>::T* __restrict__ yb,
                                                  typename Cplx<R>::T* __restrict__ xb, typename Cplx<R>::T* sig,
                                                  typename Cplx<R>::T* tt) {
  typedef typename Cplx<R>::T C;
  constexpr int NC = NB / CG;
  extern __shared__ unsigned char smem_raw[];
  const int wb = L.wb, kv = solve_kvb(L), nt = blockDim.x, tid = threadIdx.x, nblk = L.nblk;
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + wb;
  const int slot = blockIdx.x;
  const int o = phase == 1 ? (int)blockIdx.y : (int)blockIdx.y + 1;
  const int p = pl.np - 1 - o;  // runs are taken from the last block down
  const int b0 = p * pl.bpp, b1 = min(b0 + pl.bpp, nblk);
  const bool outs = phase == 3 || o == 0;
  const Entry e = ent[slot];
  const FaceTab F = ft[e.s];
  const double2* gin = e.src ? io.g_b : io.g_a;
  if (gin) gin += (size_t)e.rhs * g.nif;
  const int lo = b0 * NB, hi = min(b1 * NB, g.nloc), nedge = 2 * g.snx + 2 * (g.sny - 2);
  if (io.nz && !io.nz[(size_t)e.rhs * g.n1 * g.n2 + e.s]) {  // zero right-hand side: x = 0
    if (io.nz_skip_out || !outs) return;
    if (io.u || io.x64)
      for (int l = lo + tid; l < hi; l += nt) emit_field(g, e, io, slot, l, mk(0.0, 0.0));
    if (io.tr_dst)
      for (int q = tid; q < nedge; q += nt) {
        const int l = edge_row(g, q);
        if (l >= lo && l < hi) emit_traces(g, e, F, coef, io, gin, l, mk(0.0, 0.0));
      }
    return;
  }
  const int ylen = nblk * NB;
  const C* y = yb + (size_t)slot * ylen;
  C* x = xb + (size_t)slot * ylen;
  const C* M = MB + (size_t)e.s * L.mb_per_sub;
  const int cg = tid % CG, r = tid / CG;
  const bool act = r < wb;
  const size_t bstride = (size_t)NB * wb;
  const int kstride = wb * CG, toff = act ? r * CG + cg : 0;
  const int frow = min(tid, NB - 1);
  {
    const C* tin = tt + ((size_t)slot * pl.np + o) * pl.ns;
    for (int q = tid; q < wb; q += nt) {
      const int row = (b1 - 1) * NB - kv + q;
      C v = row >= 0 ? y[row] : czero<C>();
      if (q >= NB && o > 0) v = phase == 3 ? tin[q - NB] : czero<C>();
      bufA[q] = v;
    }
  }
  C mr[D][NC];
  C fr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const C* Mb = M + (size_t)max(b1 - 1 - d, b0) * bstride + toff;
#pragma unroll
    for (int k = 0; k < NC; ++k) mr[d][k] = Mb[k * kstride];
    fr[d] = y[max((b1 - 2 - d) * NB - kv + frow, 0)];
  }
  __syncthreads();

  auto step = [&](int b, C(&m)[NC], C& f) {
    if (tid < NB) bufB[tid] = ((b - 1) * NB - kv + tid >= 0) ? f : czero<C>();
    C acc = czero<C>();
#pragma unroll
    for (int k = 0; k < NC; ++k) cfma(acc, m[k], bufA[kv + cg * NC + k]);
    acc = row_reduce<CG>(acc);
    {
      const C* Mb = M + (size_t)max(b - D, b0) * bstride + toff;
#pragma unroll
      for (int k = 0; k < NC; ++k) m[k] = Mb[k * kstride];
      f = y[max((b - D - 1) * NB - kv + frow, 0)];
    }
    if (act && cg == 0) {
      if (r >= kv) {
        if (outs) x[b * NB + r - kv] = acc;
      } else {
        bufB[r + NB] = cadd(acc, bufA[r]);
      }
    }
    __syncthreads();
    C* t = bufA;
    bufA = bufB;
    bufB = t;
  };
  const int n = b1 - b0, nmain = (n / D) * D;
  for (int i0 = 0; i0 < nmain; i0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) step(b1 - 1 - (i0 + d), mr[d], fr[d]);
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (nmain + d < n) step(b1 - 1 - (nmain + d), mr[d], fr[d]);
  if (phase == 1) {  // the outgoing state: window rows [nb, wb) of block b0 - 1
    C* dst = o == 0 ? tt + ((size_t)slot * pl.np + 1) * pl.ns : sig + ((size_t)slot * pl.np + o) * pl.ns;
    for (int q = NB + tid; q < wb; q += nt) dst[q - NB] = bufA[q];
    if (o >= 1 && o + 1 <= pl.np - 1) {  // the chain's output state o + 1 starts unset
      C u;
      set_unset(u);
      for (int q = tid; q < kv; q += nt) tt[((size_t)slot * pl.np + o + 1) * pl.ns + q] = u;
    }
  }
  if (!outs) return;
  // this run's rows are final: their outputs, as k_bwd writes them
  if (io.u || io.x64)
    for (int l = lo + tid; l < hi; l += nt) emit_field(g, e, io, slot, l, to_d(x[l]));
  if (io.tr_dst)
    for (int q = tid; q < nedge; q += nt) {
      const int l = edge_row(g, q);
      if (l >= lo && l < hi) emit_traces(g, e, F, coef, io, gin, l, to_d(x[l]));
    }
}

// The chain: tt[o + 1] = sig[o] + Phi_o tt[o] for o = 1 .. np - 2 and every entry.  Each step's
// product is split into tasks of kChainRows rows of tt[o + 1].  The persistent workgroups of an
// entry (blockIdx.x % nent) claim its tasks from the entry's ticket counter in step order (a
// single counter for all entries made the claims contend).  A task first loads its rows of Phi_o
// (they depend on no data), then reads tt[o] until none of its entries holds the unset mark (the
// first pass marks the states o >= 2 unset; the tasks of step o - 1 overwrite them), and
// publishes its rows.  The data carry their own readiness: a completion counter per step cost a
// store wait and a counter round trip more per step (44 against 33 us forward, 59 against 42 us
// backward, per batch of 8 solves of 128^2 subdomains).
// A task only reads data of tasks of its entry with smaller tickets, claimed by workgroups that are
// running, so the launch completes whatever the number of resident workgroups; every wait is
// bounded (past spin_limit polls the error flag is set and the task goes on).  The states that
// tasks of one launch exchange are written and read with device-coherent accesses, a complex128
// entry as two 64-bit halves (both are checked).
constexpr int kPartStateMax = 576, kChainRows = 16, kChainThreads = 256, kChainU = 16;
constexpr int kChainStateRegs = (kPartStateMax + kChainThreads - 1) / kChainThreads;  // state entries per thread

__device__ inline void st_coh(double2* p, double2 v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)__double_as_longlong(v.y), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double2 ld_coh(const double2* p) {
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return mk(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
}
__device__ inline void st_coh(float2* p, float2 v) {
  const unsigned long long b = (unsigned long long)(unsigned)__float_as_int(v.x) |
                               ((unsigned long long)(unsigned)__float_as_int(v.y) << 32);
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float2 ld_coh(const float2* p) {
  const unsigned long long b =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_float2(__int_as_float((int)(unsigned)(b & 0xffffffffull)), __int_as_float((int)(unsigned)(b >> 32)));
}

template <typename C>
__global__ __launch_bounds__(kChainThreads) void k_part_chain(Geom g, PartLayout pl, int S, const Entry* ent,
                                                              int nent, const int32_t* __restrict__ nzf,
                                                              const C* __restrict__ phi, const C* sig, C* tt,
                                                              int32_t* ctr, int32_t* ctr_next, int nctr, int32_t* err,
                                                              int spin_limit) {
  // the other counter region is zeroed here for the next launch (it is not used by this one)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nctr; i += gridDim.x * blockDim.x) ctr_next[i] = 0;
  constexpr int NG = kChainThreads / kChainRows;  // column groups
  __shared__ int s_ticket;
  __shared__ C ts[kPartStateMax];
  __shared__ C red[kChainThreads];
  const int tid = threadIdx.x, ri = tid % kChainRows, jg = tid / kChainRows;
  const int W = (S + kChainRows - 1) / kChainRows;  // tasks per step and entry
  const int ntasks = (pl.np - 2) * W;               // per entry
  const int slot = blockIdx.x % nent;
  for (;;) {
    // uniform loop: the ticket goes through LDS and is read back as a scalar
    __syncthreads();  // the previous task no longer reads s_ticket, ts or red
    if (tid == 0) s_ticket = __hip_atomic_fetch_add(ctr + slot, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t < 0 || t >= ntasks) break;
    const int o = 1 + t / W, w = t - (o - 1) * W;
    const Entry e = ent[slot];
    const bool live = !(nzf && !nzf[(size_t)e.rhs * g.n1 * g.n2 + e.s]);
    const int i = w * kChainRows + ri;
    const bool rowok = i < S;
    // 1. this task's rows of Phi_o, the first kChainU columns of each group (independent of the data)
    const C* F = phi + ((size_t)e.s * (pl.np - 2) + (o - 1)) * S * S;
    C f[kChainU];
#pragma unroll
    for (int u = 0; u < kChainU; ++u) {
      const int j = jg + NG * u;
      f[u] = (live && rowok && j < S) ? F[(size_t)j * S + i] : czero<C>();
    }
    // 2. tt[o] (written by the tasks of step o - 1 of this entry, or by the first pass for o = 1),
    //    read until no entry is unset, into LDS
    if (live) {
      const C* src = tt + ((size_t)slot * pl.np + o) * pl.ns;
      C v[kChainStateRegs];
      for (int polls = 0;; ++polls) {
        int miss = 0;
#pragma unroll
        for (int r = 0; r < kChainStateRegs; ++r) {
          const int q = tid + r * kChainThreads;
          if (q < S) {
            v[r] = ld_coh(src + q);
            miss |= is_unset(v[r]);
          }
        }
        if (!__syncthreads_or(miss)) break;
        if (polls >= spin_limit) {
          if (tid == 0) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
#pragma unroll
      for (int r = 0; r < kChainStateRegs; ++r) {
        const int q = tid + r * kChainThreads;
        if (q < S) ts[q] = v[r];
      }
    }
    __syncthreads();
    C acc = czero<C>();
    if (live) {
#pragma unroll
      for (int u = 0; u < kChainU; ++u) {
        const int j = jg + NG * u;
        if (j < S) cfma(acc, f[u], ts[j]);
      }
      for (int j0 = NG * kChainU; j0 < S; j0 += NG * kChainU) {  // windows wider than 256 rows
#pragma unroll
        for (int u = 0; u < kChainU; ++u) {
          const int j = j0 + jg + NG * u;
          if (rowok && j < S) cfma(acc, F[(size_t)j * S + i], ts[j]);
        }
      }
    }
    red[tid] = acc;
    __syncthreads();
    // 4. publish the rows (their values mark them written)
    if (tid < kChainRows && live && rowok) {
      C v = sig[((size_t)slot * pl.np + o) * pl.ns + i];
      for (int q = 0; q < NG; ++q) v = cadd(v, red[q * kChainRows + tid]);
      st_coh(tt + ((size_t)slot * pl.np + o + 1) * pl.ns + i, v);
    }
  }
}

// Transfer matrices of the forward runs 1 .. np - 2: workgroup (column group, run, subdomain)
// carries NCOL unit incoming states through the run's blocks with no right-hand side (the window
// [wf][NCOL] in LDS, twice for the row interchanges; thread i owns state row i), then stores the
// outgoing states as columns.
template <typename C, int NCOL>
__global__ __launch_bounds__(576) void k_part_phi_fwd(Geom g, SolveLayout L, PartLayout pl,
                                                      const C* __restrict__ MF, const int16_t* __restrict__ PF,
                                                      const int32_t* __restrict__ PFL, C* __restrict__ phi) {
  constexpr int NB = 16;
  extern __shared__ unsigned char smem_raw[];
  const int wf = L.wf, kl = g.kl, nblk = L.nblk, tid = threadIdx.x, nt = blockDim.x, cgf = L.cgf;
  C* win = reinterpret_cast<C*>(smem_raw);  // [wf][NCOL]
  C* alt = win + (size_t)wf * NCOL;         // the same, for the interchanges
  const int s = blockIdx.z, o = blockIdx.y + 1, c0 = blockIdx.x * NCOL;
  const int b0 = o * pl.bpp, b1 = min(b0 + pl.bpp, nblk);
  const C* M = MF + (size_t)s * L.mf_per_sub;
  const int16_t* P = PF + (size_t)s * L.pf_per_sub;
  const int32_t* PI = PFL + (size_t)s * nblk;
  C one = czero<C>();
  one.x = 1;
  for (int idx = tid; idx < wf * NCOL; idx += nt) {
    const int q = idx / NCOL, c = idx - q * NCOL;
    win[idx] = (q < kl && q == c0 + c) ? one : czero<C>();
  }
  __syncthreads();
  const bool act = tid < kl;
  const int r = NB + (act ? tid : 0);  // the window row this thread updates
  for (int b = b0; b < b1; ++b) {
    if (!PI[b]) {  // row interchanges inside this block's window
      const int16_t* Pb = P + (size_t)b * wf;
      for (int idx = tid; idx < wf * NCOL; idx += nt) {
        const int q = idx / NCOL, c = idx - q * NCOL;
        alt[idx] = win[(int)Pb[q] * NCOL + c];
      }
      __syncthreads();
      C* t = win;
      win = alt;
      alt = t;
    }
    C acc[NCOL];
    if (act) {
      const C* Mb = M + (size_t)b * NB * wf;
      C m[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) m[k] = Mb[tile_index(k, r, wf, NB, cgf)];
#pragma unroll
      for (int c = 0; c < NCOL; ++c) acc[c] = win[r * NCOL + c];
#pragma unroll
      for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int c = 0; c < NCOL; ++c) cfma(acc[c], m[k], win[k * NCOL + c]);
    }
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < NCOL; ++c) win[tid * NCOL + c] = acc[c];
    if (tid < NB)
#pragma unroll
      for (int c = 0; c < NCOL; ++c) win[(kl + tid) * NCOL + c] = czero<C>();
    __syncthreads();
  }
  if (act) {
    C* F = phi + ((size_t)s * (pl.np - 2) + (o - 1)) * kl * kl;
#pragma unroll
    for (int c = 0; c < NCOL; ++c)
      if (c0 + c < kl) F[(size_t)(c0 + c) * kl + tid] = win[tid * NCOL + c];
  }
}

// Transfer matrices of the backward runs 1 .. np - 2 (run o covers the blocks of partition
// np - 1 - o, taken from its last block down); window [wb][NCOL], state rows [nb, wb).
template <typename C, int NCOL>
__global__ __launch_bounds__(576) void k_part_phi_bwd(Geom g, SolveLayout L, PartLayout pl,
                                                      const C* __restrict__ MB, C* __restrict__ phi) {
  constexpr int NB = 16;
  extern __shared__ unsigned char smem_raw[];
  C* win = reinterpret_cast<C*>(smem_raw);  // [wb][NCOL]
  const int wb = L.wb, kv = solve_kvb(L), nblk = L.nblk, tid = threadIdx.x, nt = blockDim.x, cgb = L.cgb;
  const int s = blockIdx.z, o = blockIdx.y + 1, c0 = blockIdx.x * NCOL;
  const int p = pl.np - 1 - o;
  const int b0 = p * pl.bpp, b1 = min(b0 + pl.bpp, nblk);
  const C* M = MB + (size_t)s * L.mb_per_sub;
  C one = czero<C>();
  one.x = 1;
  for (int idx = tid; idx < wb * NCOL; idx += nt) {
    const int q = idx / NCOL, c = idx - q * NCOL;
    win[idx] = (q >= NB && q - NB == c0 + c) ? one : czero<C>();
  }
  __syncthreads();
  const bool act = tid < kv;
  const int r = act ? tid : 0;
  for (int b = b1 - 1; b >= b0; --b) {
    C acc[NCOL];
    if (act) {
      const C* Mb = M + (size_t)b * NB * wb;
      C m[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) m[k] = Mb[tile_index(k, r, wb, NB, cgb)];
#pragma unroll
      for (int c = 0; c < NCOL; ++c) acc[c] = win[r * NCOL + c];
#pragma unroll
      for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int c = 0; c < NCOL; ++c) cfma(acc[c], m[k], win[(kv + k) * NCOL + c]);
    }
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < NCOL; ++c) win[(tid + NB) * NCOL + c] = acc[c];
    if (tid < NB)
#pragma unroll
      for (int c = 0; c < NCOL; ++c) win[tid * NCOL + c] = czero<C>();
    __syncthreads();
  }
  if (act) {
    C* F = phi + ((size_t)s * (pl.np - 2) + (o - 1)) * kv * kv;
#pragma unroll
    for (int c = 0; c < NCOL; ++c)
      if (c0 + c < kv) F[(size_t)(c0 + c) * kv + tid] = win[(NB + tid) * NCOL + c];
  }
}

}  // namespace

// column groups per window row (must match the tiled layout written by the repack)
void solve_column_groups(int wf, int wb, int* cgf, int* cgb) {
  *cgf = (wf * 4 <= 576) ? 4 : 1;
  *cgb = (wb * 2 <= 576) ? 2 : 1;
}

// Register prefetch depth (column blocks in flight per lane) of the one-workgroup-per-solve
// kernels, per precision and depth variant; variant 0 is the default, the autotuner times the
// others.  Every depth keeps the kernels within the registers of three wavefronts per SIMD (the
// 576-thread workgroup) without spills: the complex128 backward kernel has no third depth (at 4
// it spills), so its variant 2 repeats the default.
constexpr int kFwdDepth[2][kSolveDepthVariants] = {{5, 3, 6}, {8, 4, 10}};  // [double, float]
constexpr int kBwdDepth[2][kSolveDepthVariants] = {{3, 2, 3}, {4, 3, 6}};

int solve_depth(bool fwd, size_t real_bytes, int dv) {
  if (dv < 0 || dv >= kSolveDepthVariants) dv = 0;
  return (fwd ? kFwdDepth : kBwdDepth)[real_bytes == 8 ? 0 : 1][dv];
}

template <typename R>
hipError_t launch_fwd(const Geom& g, const SolveLayout& L, const Entry* ent, int nent, const FaceTab* ft,
                      const IfCoef* coef, const typename Cplx<R>::T* mf, const int16_t* pf, const int32_t* pflag,
                      const SolveIO& io, typename Cplx<R>::T* ybuf, hipStream_t st, int dv) {
  typedef typename Cplx<R>::T C;
  if (nent == 0) return hipSuccess;
  if (L.nb != 16 || L.wf > 576) return hipErrorInvalidValue;
  const size_t shm = 2 * (size_t)L.wf * sizeof(C) + (size_t)L.nblk * sizeof(int);
  const int rows = L.wf * L.cgf;
  const dim3 blk(((rows + 63) / 64) * 64);
#define HBJ_FWD(CG, D) \
  hipLaunchKernelGGL((k_fwd<R, 16, CG, D>), dim3(nent), blk, shm, st, g, L, ent, ft, coef, mf, pf, pflag, io, ybuf)
  if (L.cgf == 4) {
    const int d = solve_depth(true, sizeof(R), dv);
    if constexpr (sizeof(R) == 8) {
      if (d == 3) HBJ_FWD(4, 3);
      else if (d == 6) HBJ_FWD(4, 6);
      else HBJ_FWD(4, 5);
    } else {
      if (d == 4) HBJ_FWD(4, 4);
      else if (d == 10) HBJ_FWD(4, 10);
      else HBJ_FWD(4, 8);
    }
  } else {
    HBJ_FWD(1, 1);
  }
#undef HBJ_FWD
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bwd(const Geom& g, const SolveLayout& L, const Entry* ent, int nent, const FaceTab* ft,
                      const IfCoef* coef, const typename Cplx<R>::T* mb, const SolveIO& io,
                      typename Cplx<R>::T* ybuf, hipStream_t st, int dv) {
  typedef typename Cplx<R>::T C;
  if (nent == 0) return hipSuccess;
  if (L.nb != 16 || L.wb > 576) return hipErrorInvalidValue;
  const size_t shm = 2 * (size_t)L.wb * sizeof(C);
  const int rows = L.wb * L.cgb;
  const dim3 blk(((rows + 63) / 64) * 64);
#define HBJ_BWD(CG, D) \
  hipLaunchKernelGGL((k_bwd<R, 16, CG, D>), dim3(nent), blk, shm, st, g, L, ent, ft, coef, mb, io, ybuf)
  if (L.cgb == 2) {
    const int d = solve_depth(false, sizeof(R), dv);
    if constexpr (sizeof(R) == 8) {
      if (d == 2) HBJ_BWD(2, 2);
      else HBJ_BWD(2, 3);
    } else {
      if (d == 3) HBJ_BWD(2, 3);
      else if (d == 6) HBJ_BWD(2, 6);
      else HBJ_BWD(2, 4);
    }
  } else {
    HBJ_BWD(1, 1);
  }
#undef HBJ_BWD
  return hipGetLastError();
}

template hipError_t launch_fwd<double>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                       const IfCoef*, const double2*, const int16_t*, const int32_t*, const SolveIO&,
                                       double2*, hipStream_t, int);
template hipError_t launch_fwd<float>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                      const IfCoef*, const float2*, const int16_t*, const int32_t*, const SolveIO&,
                                      float2*, hipStream_t, int);
template hipError_t launch_bwd<double>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                       const IfCoef*, const double2*, const SolveIO&, double2*, hipStream_t, int);
template hipError_t launch_bwd<float>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                      const IfCoef*, const float2*, const SolveIO&, float2*, hipStream_t, int);

constexpr int kMmSpwMax = 5;  // window tiles per wavefront of the MFMA solves: windows of up to 20 tiles

// tiles per wavefront for a window of `rows` rows (the window is padded to 4 x that many tiles)
static int mm_spw(int rows) { return ((rows + 15) / 16 + 3) / 4; }

// X, flags, interchange scratch / tiles passed on and final rows
static size_t fwd_mm_lds(const SolveLayout& L, size_t elem, bool piv = true) {
  return 512 * elem + (piv ? (size_t)((L.nblk + 3) & ~3) * sizeof(int) : 0) +
         (size_t)std::max(piv ? 4 * mm_spw(L.wf) : 0, 8) * 256 * elem;
}

bool trisolve_mm_fits(const SolveLayout& L, size_t elem) {
  return L.nb == 16 && mm_spw(L.wf) <= kMmSpwMax && mm_spw(L.wb) <= kMmSpwMax && fwd_mm_lds(L, elem) <= 64 * 1024;
}

template <typename R>
hipError_t launch_fwd_mm(const Geom& g, const SolveLayout& L, const Entry* ent, const int2* tiles, int ntiles,
                         const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mf, const int16_t* pf,
                         const int32_t* pflag, bool piv, const SolveIO& io, typename Cplx<R>::T* ybuf,
                         typename Cplx<R>::T* sink, hipStream_t st) {
  typedef typename Cplx<R>::T C;
  if (ntiles == 0) return hipSuccess;
  if (!trisolve_mm_fits(L, sizeof(C))) return hipErrorInvalidValue;
  const size_t shm = fwd_mm_lds(L, sizeof(C), piv);
#define HBJ_FWD_MM(S, P)                                                                                      \
  hipLaunchKernelGGL((k_fwd_mm<R, S, P>), dim3(ntiles), dim3(256), shm, st, g, L, ent, tiles, ft, coef, mf, pf, \
                     pflag, io, ybuf, sink)
#define HBJ_FWD_MM2(S) \
  if (piv) HBJ_FWD_MM(S, true); else HBJ_FWD_MM(S, false)
  switch (mm_spw(L.wf)) {
    case 1: HBJ_FWD_MM2(1); break;
    case 2: HBJ_FWD_MM2(2); break;
    case 3: HBJ_FWD_MM2(3); break;
    case 4: HBJ_FWD_MM2(4); break;
    default: HBJ_FWD_MM2(5); break;
  }
#undef HBJ_FWD_MM2
#undef HBJ_FWD_MM
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bwd_mm(const Geom& g, const SolveLayout& L, const Entry* ent, const int2* tiles, int ntiles,
                         const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mb, const SolveIO& io,
                         typename Cplx<R>::T* ybuf, typename Cplx<R>::T* sink, hipStream_t st) {
  typedef typename Cplx<R>::T C;
  if (ntiles == 0) return hipSuccess;
  if (!trisolve_mm_fits(L, sizeof(C))) return hipErrorInvalidValue;
  const size_t shm = (512 + 8 * 256) * sizeof(C);  // X, tiles passed on, final rows
#define HBJ_BWD_MM(S)                                                                                           \
  hipLaunchKernelGGL((k_bwd_mm<R, S>), dim3(ntiles), dim3(256), shm, st, g, L, ent, tiles, ft, coef, mb, io, ybuf, \
                     sink)
  switch (mm_spw(L.wb)) {
    case 1: HBJ_BWD_MM(1); break;
    case 2: HBJ_BWD_MM(2); break;
    case 3: HBJ_BWD_MM(3); break;
    case 4: HBJ_BWD_MM(4); break;
    default: HBJ_BWD_MM(5); break;
  }
#undef HBJ_BWD_MM
  return hipGetLastError();
}

template hipError_t launch_fwd_mm<double>(const Geom&, const SolveLayout&, const Entry*, const int2*, int,
                                          const FaceTab*, const IfCoef*, const double2*, const int16_t*,
                                          const int32_t*, bool, const SolveIO&, double2*, double2*, hipStream_t);
template hipError_t launch_fwd_mm<float>(const Geom&, const SolveLayout&, const Entry*, const int2*, int,
                                         const FaceTab*, const IfCoef*, const float2*, const int16_t*, const int32_t*,
                                         bool, const SolveIO&, float2*, float2*, hipStream_t);
template hipError_t launch_bwd_mm<double>(const Geom&, const SolveLayout&, const Entry*, const int2*, int,
                                          const FaceTab*, const IfCoef*, const double2*, const SolveIO&, double2*,
                                          double2*, hipStream_t);
template hipError_t launch_bwd_mm<float>(const Geom&, const SolveLayout&, const Entry*, const int2*, int,
                                         const FaceTab*, const IfCoef*, const float2*, const SolveIO&, float2*,
                                         float2*, hipStream_t);

hipError_t launch_build_rhs(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfCoef* coef,
                            const SolveIO& io, double2* rhs64, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_rhs, dim3((g.nloc + 255) / 256, nent), dim3(256), 0, st, g, ent, ft, coef, io, rhs64);
  return hipGetLastError();
}

hipError_t launch_emit_traces(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfBand* band,
                              const SolveIO& io, const double2* x64, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_emit_traces, dim3((g.nloc + 255) / 256, nent), dim3(256), 0, st, g, ent, ft, band, io, x64);
  return hipGetLastError();
}

hipError_t launch_axpy_c64(double2* x64, const float2* dx, const Geom& g, const SolveLayout& L, int nent,
                           hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_c64, dim3((g.nloc + 255) / 256, nent), dim3(256), 0, st, x64, dx, g.nloc,
                     L.nblk * L.nb);
  return hipGetLastError();
}

hipError_t launch_source_flags(const Geom& g, const double2* f, int nrhs, int32_t* nz, hipStream_t st) {
  hipLaunchKernelGGL(k_source_flags, dim3(g.n1 * g.n2, nrhs), dim3(kFlagThreads), 0, st, g, f, nz);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// partitioned solves
bool part_fits(const Geom& g, const SolveLayout& L) {
  // the windows of the transfer-matrix kernels (the forward one twice, 4 columns at least) within 64 KiB
  return L.nb == 16 && L.wf <= 576 && L.wb <= 576 && solve_kvb(L) <= kPartStateMax && g.kl <= kPartStateMax &&
         2 * L.wf * 4 * sizeof(double2) <= 65536 && L.wb * 4 * sizeof(double2) <= 65536;
}

template <typename C>
static int part_ncol(int rows) {  // columns of a transfer-matrix workgroup: the window within 64 KiB of LDS
  return rows * 16 * (int)sizeof(C) <= 65536 ? 16 : rows * 8 * (int)sizeof(C) <= 65536 ? 8 : 4;
}

template <typename R>
hipError_t launch_part_phi(const Geom& g, const SolveLayout& L, const PartLayout& pl,
                           const typename Cplx<R>::T* mf, const int16_t* pf, const int32_t* pflag,
                           const typename Cplx<R>::T* mb, typename Cplx<R>::T* phi_f, typename Cplx<R>::T* phi_b,
                           int nsub, hipStream_t st) {
  typedef typename Cplx<R>::T C;
  if (pl.np <= 2 || nsub == 0) return hipSuccess;
  if (!part_fits(g, L)) return hipErrorInvalidValue;
  {
    const int nc = part_ncol<C>(2 * L.wf);
    const dim3 grid((g.kl + nc - 1) / nc, pl.np - 2, nsub), blk(((g.kl + 63) / 64) * 64);
    const size_t shm = 2 * (size_t)L.wf * nc * sizeof(C);
    if (nc == 16) hipLaunchKernelGGL((k_part_phi_fwd<C, 16>), grid, blk, shm, st, g, L, pl, mf, pf, pflag, phi_f);
    else if (nc == 8) hipLaunchKernelGGL((k_part_phi_fwd<C, 8>), grid, blk, shm, st, g, L, pl, mf, pf, pflag, phi_f);
    else hipLaunchKernelGGL((k_part_phi_fwd<C, 4>), grid, blk, shm, st, g, L, pl, mf, pf, pflag, phi_f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const int nc = part_ncol<C>(L.wb);
    const int kvb = solve_kvb(L);
    const dim3 grid((kvb + nc - 1) / nc, pl.np - 2, nsub), blk(((kvb + 63) / 64) * 64);
    const size_t shm = (size_t)L.wb * nc * sizeof(C);
    if (nc == 16) hipLaunchKernelGGL((k_part_phi_bwd<C, 16>), grid, blk, shm, st, g, L, pl, mb, phi_b);
    else if (nc == 8) hipLaunchKernelGGL((k_part_phi_bwd<C, 8>), grid, blk, shm, st, g, L, pl, mb, phi_b);
    else hipLaunchKernelGGL((k_part_phi_bwd<C, 4>), grid, blk, shm, st, g, L, pl, mb, phi_b);
  }
  return hipGetLastError();
}

int part_chain_counters(int nent, int np) {
  (void)np;  // one ticket counter per entry, whatever the run count
  return nent;
}

// one chain launch: counters of region pw.parity (zeroed by the previous launch or at allocation),
// the other region zeroed for the next one; per entry, workgroups for two steps' tasks
template <typename C>
static hipError_t launch_chain(const Geom& g, const PartLayout& pl, int S, const Entry* ent, int nent,
                               const int32_t* nz, const C* phi, const C* sig, C* tt, PartWait& pw, hipStream_t st) {
  if (S > kPartStateMax || pw.nctr < part_chain_counters(nent, pl.np)) return hipErrorInvalidValue;
  const int W = (S + kChainRows - 1) / kChainRows;
  const int per = std::max(1, std::min(std::min((pl.np - 2) * W, 2 * W), kChainGridMax / std::max(nent, 1)));
  const int grid = nent * per;
  int32_t* cur = pw.ctr + (size_t)pw.parity * pw.nctr;
  int32_t* nxt = pw.ctr + (size_t)(1 - pw.parity) * pw.nctr;
  hipLaunchKernelGGL(k_part_chain<C>, dim3(grid), dim3(kChainThreads), 0, st, g, pl, S, ent, nent, nz, phi, sig, tt,
                     cur, nxt, pw.nctr, pw.err, pw.spin);
  pw.parity ^= 1;
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fwd_part(const Geom& g, const SolveLayout& L, const PartLayout& pl, const Entry* ent, int nent,
                           const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mf, const int16_t* pf,
                           const int32_t* pflag, const typename Cplx<R>::T* phi_f, const SolveIO& io,
                           typename Cplx<R>::T* rb, typename Cplx<R>::T* y2, typename Cplx<R>::T* sig,
                           typename Cplx<R>::T* tt, PartWait& pw, hipStream_t st) {
  typedef typename Cplx<R>::T C;
  if (nent == 0) return hipSuccess;
  if (!part_fits(g, L) || pl.np < 2 || pl.bpp < 1 || (pl.np - 1) * pl.bpp >= L.nblk || pl.ns < solve_kvb(L))
    return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  const size_t shm = 2 * (size_t)L.wf * sizeof(C) + (size_t)pl.bpp * sizeof(int);
  const dim3 blk(((L.wf * L.cgf + 63) / 64) * 64);
  for (int phase = 1; phase <= 3; phase += 2) {
    const dim3 grid(nent, phase == 1 ? pl.np : pl.np - 1);  // pass 1: also the last run's right-hand side
#define HBJ_FWDP(CG, D)                                                                                         \
  hipLaunchKernelGGL((k_fwd_part<R, 16, CG, D>), grid, blk, shm, st, g, L, pl, phase, ent, ft, coef, io, mf, pf, \
                     pflag, rb, y2, sig, tt)
    if (L.cgf == 4) {
      if constexpr (sizeof(R) == 8) HBJ_FWDP(4, 5);
      else HBJ_FWDP(4, 8);
    } else {
      HBJ_FWDP(1, 1);
    }
#undef HBJ_FWDP
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (phase == 1 && pl.np > 2) {
      e = launch_chain<C>(g, pl, g.kl, ent, nent, io.nz, phi_f, sig, tt, pw, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename R>
hipError_t launch_bwd_part(const Geom& g, const SolveLayout& L, const PartLayout& pl, const Entry* ent, int nent,
                           const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mb,
                           const typename Cplx<R>::T* phi_b, const SolveIO& io, const typename Cplx<R>::T* y2,
                           typename Cplx<R>::T* rb, typename Cplx<R>::T* sig, typename Cplx<R>::T* tt, PartWait& pw,
                           hipStream_t st) {
  typedef typename Cplx<R>::T C;
  if (nent == 0) return hipSuccess;
  if (!part_fits(g, L) || pl.np < 2 || pl.bpp < 1 || (pl.np - 1) * pl.bpp >= L.nblk || pl.ns < solve_kvb(L))
    return hipErrorInvalidValue;
  const size_t shm = 2 * (size_t)L.wb * sizeof(C);
  const dim3 grid(nent, pl.np - 1), blk(((L.wb * L.cgb + 63) / 64) * 64);
  hipError_t e = hipSuccess;
  for (int phase = 1; phase <= 3; phase += 2) {
#define HBJ_BWDP(CG, D)                                                                                            \
  hipLaunchKernelGGL((k_bwd_part<R, 16, CG, D>), grid, blk, shm, st, g, L, pl, phase, ent, ft, coef, mb, io, y2, rb, \
                     sig, tt)
    if (L.cgb == 2) {
      if constexpr (sizeof(R) == 8) HBJ_BWDP(2, 3);
      else HBJ_BWDP(2, 4);
    } else {
      HBJ_BWDP(1, 1);
    }
#undef HBJ_BWDP
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (phase == 1 && pl.np > 2) {
      e = launch_chain<C>(g, pl, solve_kvb(L), ent, nent, io.nz, phi_b, sig, tt, pw, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

#define HBJ_PART_INST(R, C)                                                                                      \
  template hipError_t launch_part_phi<R>(const Geom&, const SolveLayout&, const PartLayout&, const C*, const int16_t*, \
                                         const int32_t*, const C*, C*, C*, int, hipStream_t);                        \
  template hipError_t launch_fwd_part<R>(const Geom&, const SolveLayout&, const PartLayout&, const Entry*, int,        \
                                         const FaceTab*, const IfCoef*, const C*, const int16_t*, const int32_t*,      \
                                         const C*, const SolveIO&, C*, C*, C*, C*, PartWait&, hipStream_t);           \
  template hipError_t launch_bwd_part<R>(const Geom&, const SolveLayout&, const PartLayout&, const Entry*, int,        \
                                         const FaceTab*, const IfCoef*, const C*, const C*, const SolveIO&, const C*,  \
                                         C*, C*, C*, PartWait&, hipStream_t);
HBJ_PART_INST(double, double2)
HBJ_PART_INST(float, float2)
#undef HBJ_PART_INST
