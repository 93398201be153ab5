// Batched single-right-hand-side triangular solves with the repacked band LU factors.
//
// Each workgroup performs one local solve u = A_s^{-1} rhs (the unit of work of every
// interface operator, paper Sec. 4).  The forward solve keeps a window of
// wf = nb + kl rows of the right-hand side in LDS; per column block it gathers the
// window through the block's interchange permutation and applies the
// (nb + kl) x nb matrix Mf: the first nb rows are final, the remaining kl rows
// slide down and nb fresh rows enter.  The backward solve walks the blocks from
// the last one with a window of kv + nb rows (kv = kl + ku, the bandwidth of U).
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

// Final value x of local row l: write it where the launch asks for it.
__device__ inline void emit(const Geom& g, const Entry& e, const FaceTab& F, const IfCoef* coef, const SolveIO& io,
                            const double2* gin, int slot, int l, double2 x) {
  if (l >= g.nloc) return;
  if (io.x64) io.x64[(size_t)slot * g.nloc + l] = x;
  const int ly = l / g.snx, lx = l - ly * g.snx;
  if (io.u) {
    const int x0 = (e.s % g.n1) * g.snx, y0 = (e.s / g.n1) * g.sny;
    io.u[(size_t)e.rhs * g.nx * g.ny + (size_t)(y0 + ly) * g.nx + x0 + lx] = x;
  }
  if (io.tr_dst) {
    const bool on[4] = {lx == 0, lx == g.snx - 1, ly == 0, ly == g.sny - 1};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (!on[f] || !((e.mask >> f) & 1) || F.out_off[f] < 0) continue;
      const int ee = (f < 2) ? ly : lx;
      const int qi = F.in_off[f] + ee, qo = F.out_off[f] + ee;
      const IfCoef c = coef[qi];
      double2 val = cmul(c.sigma, x);
      if (io.tr_reflect && gin) cfma(val, c.rho, gin[qi]);
      // out = -rho g - sigma u
      val = mk(-val.x, -val.y);
      const size_t o = (size_t)e.rhs * g.nif + qo;
      double2 base = io.tr_base ? io.tr_base[o] : mk(0.0, 0.0);
      base.x += io.tr_sign * val.x;
      base.y += io.tr_sign * val.y;
      io.tr_dst[o] = base;
    }
  }
}

template <typename R, int NB>
__global__ __launch_bounds__(320) void k_fwd(Geom g, SolveLayout L, const Entry* ent, const FaceTab* ft,
                                             const IfCoef* coef, const typename Cplx<R>::T* __restrict__ MF,
                                             const int16_t* __restrict__ PF, SolveIO io,
                                             typename Cplx<R>::T* __restrict__ ybuf) {
  typedef typename Cplx<R>::T C;
  extern __shared__ unsigned char smem_raw[];
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + L.wf;
  const Entry e = ent[blockIdx.x];
  const FaceTab F = ft[e.s];
  const RhsCtx rhs(g, e, F, coef, io, blockIdx.x);
  const C* M = MF + (size_t)e.s * L.mf_per_sub;
  const int16_t* P = PF + (size_t)e.s * L.pf_per_sub;
  C* y = ybuf + (size_t)blockIdx.x * L.nblk * NB;
  const int wf = L.wf, kl = g.kl, nt = blockDim.x, tid = threadIdx.x;

  for (int r = tid; r < wf; r += nt) bufA[r] = to_c<C>(rhs(r));
  __syncthreads();
  for (int b = 0; b < L.nblk; ++b) {
    const C* Mb = M + (size_t)b * NB * wf;
    const int16_t* Pb = P + (size_t)b * wf;
    C t[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) t[c] = bufA[Pb[c]];
    for (int r = tid; r < wf; r += nt) {
      C acc = (r >= NB) ? bufA[Pb[r]] : czero<C>();
#pragma unroll
      for (int c = 0; c < NB; ++c) cfma(acc, Mb[(size_t)c * wf + r], t[c]);
      if (r < NB) y[b * NB + r] = acc;
      else bufB[r - NB] = acc;
    }
    for (int i = tid; i < NB; i += nt) bufB[kl + i] = to_c<C>(rhs((b + 1) * NB + kl + i));
    __syncthreads();
    C* tmp = bufA;
    bufA = bufB;
    bufB = tmp;
  }
}

template <typename R, int NB>
__global__ __launch_bounds__(320) void k_bwd(Geom g, SolveLayout L, const Entry* ent, const FaceTab* ft,
                                             const IfCoef* coef, const typename Cplx<R>::T* __restrict__ MB,
                                             SolveIO io, typename Cplx<R>::T* __restrict__ ybuf) {
  typedef typename Cplx<R>::T C;
  extern __shared__ unsigned char smem_raw[];
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + L.wb;
  const Entry e = ent[blockIdx.x];
  const FaceTab F = ft[e.s];
  const C* M = MB + (size_t)e.s * L.mb_per_sub;
  C* y = ybuf + (size_t)blockIdx.x * L.nblk * NB;
  const double2* gin = e.src ? io.g_b : io.g_a;
  if (gin) gin += (size_t)e.rhs * g.nif;
  const int wb = L.wb, kv = g.kv, nt = blockDim.x, tid = threadIdx.x;

  int j0 = (L.nblk - 1) * NB;
  for (int q = tid; q < wb; q += nt) {
    const int row = j0 - kv + q;
    bufA[q] = (row >= 0) ? y[row] : czero<C>();
  }
  __syncthreads();
  for (int b = L.nblk - 1; b >= 0; --b) {
    j0 = b * NB;
    const C* Mb = M + (size_t)b * NB * wb;
    C t[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) t[c] = bufA[kv + c];
    for (int q = tid; q < wb; q += nt) {
      C acc = (q < kv) ? bufA[q] : czero<C>();
#pragma unroll
      for (int c = 0; c < NB; ++c) cfma(acc, Mb[(size_t)c * wb + q], t[c]);
      if (q >= kv) {
        const int row = j0 + q - kv;
        y[row] = acc;
        emit(g, e, F, coef, io, gin, blockIdx.x, row, to_d(acc));
      } else {
        bufB[q + NB] = acc;
      }
    }
    for (int i = tid; i < NB; i += nt) {
      const int row = j0 - NB - kv + i;
      bufB[i] = (row >= 0) ? y[row] : czero<C>();
    }
    __syncthreads();
    C* tmp = bufA;
    bufA = bufB;
    bufB = tmp;
  }
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
__global__ void k_emit_traces(Geom g, const Entry* ent, const FaceTab* ft, const IfCoef* coef, SolveIO io,
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
  emit(g, e, F, coef, io, gin, slot, l, x64[(size_t)slot * g.nloc + l]);
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

inline int threads_for(int rows) {
  int t = ((rows + 63) / 64) * 64;
  return t > 320 ? 320 : t;
}

}  // namespace

template <typename R>
hipError_t launch_fwd(const Geom& g, const SolveLayout& L, const Entry* ent, int nent, const FaceTab* ft,
                      const IfCoef* coef, const typename Cplx<R>::T* mf, const int16_t* pf, const SolveIO& io,
                      typename Cplx<R>::T* ybuf, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  if (L.nb != 32) return hipErrorInvalidValue;
  const size_t shm = 2 * (size_t)L.wf * sizeof(typename Cplx<R>::T);
  hipLaunchKernelGGL((k_fwd<R, 32>), dim3(nent), dim3(threads_for(L.wf)), shm, st, g, L, ent, ft, coef, mf, pf, io,
                     ybuf);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bwd(const Geom& g, const SolveLayout& L, const Entry* ent, int nent, const FaceTab* ft,
                      const IfCoef* coef, const typename Cplx<R>::T* mb, const SolveIO& io,
                      typename Cplx<R>::T* ybuf, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  if (L.nb != 32) return hipErrorInvalidValue;
  const size_t shm = 2 * (size_t)L.wb * sizeof(typename Cplx<R>::T);
  hipLaunchKernelGGL((k_bwd<R, 32>), dim3(nent), dim3(threads_for(L.wb)), shm, st, g, L, ent, ft, coef, mb, io,
                     ybuf);
  return hipGetLastError();
}

template hipError_t launch_fwd<double>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                       const IfCoef*, const double2*, const int16_t*, const SolveIO&, double2*,
                                       hipStream_t);
template hipError_t launch_fwd<float>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                      const IfCoef*, const float2*, const int16_t*, const SolveIO&, float2*,
                                      hipStream_t);
template hipError_t launch_bwd<double>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                       const IfCoef*, const double2*, const SolveIO&, double2*, hipStream_t);
template hipError_t launch_bwd<float>(const Geom&, const SolveLayout&, const Entry*, int, const FaceTab*,
                                      const IfCoef*, const float2*, const SolveIO&, float2*, hipStream_t);

hipError_t launch_build_rhs(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfCoef* coef,
                            const SolveIO& io, double2* rhs64, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_rhs, dim3((g.nloc + 255) / 256, nent), dim3(256), 0, st, g, ent, ft, coef, io, rhs64);
  return hipGetLastError();
}

hipError_t launch_emit_traces(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfCoef* coef,
                              const SolveIO& io, const double2* x64, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_emit_traces, dim3((g.nloc + 255) / 256, nent), dim3(256), 0, st, g, ent, ft, coef, io, x64);
  return hipGetLastError();
}

hipError_t launch_axpy_c64(double2* x64, const float2* dx, const Geom& g, const SolveLayout& L, int nent,
                           hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_c64, dim3((g.nloc + 255) / 256, nent), dim3(256), 0, st, x64, dx, g.nloc,
                     L.nblk * L.nb);
  return hipGetLastError();
}
