// Dense local scattering operators (paper Sec. 4, the operators S_{m(j,i), m(i,k)}).
// Storage: blocks of 8 rows, T[s][row / 8][col][row % 8] (t_index), L x L per subdomain.
//
// For subdomain s the map from its incoming Robin data (all faces, local interface
// order W, E, S, N) to its outgoing data is linear:
//   out = T_s g,   T_s = -diag(rho) - diag(sigma) R A_s^{-1} B
// with B the injection g / (beta- h^2) on the edge rows and R the restriction to the
// edge nodes.  Column c of T_s is built from one local solve with a unit datum at
// position c.  Applying T_s is then a dense matrix-vector product whose rows can be
// spread over many workgroups, instead of one workgroup walking the whole band.
#include <hip/hip_ext.h>

#include <type_traits>

#include "hbj_internal.h"

namespace {

// Column e.rhs of T_s for every entry (s, col): x = A_s^{-1} B e_col is in ybuf[entry].  The
// datum sent at the row's face entry ee is -sum_d R[ee][ee+d] g - sum_d Sigma[ee][ee+d] x along
// that face (first order: -rho g - sigma x at ee only), with g the unit datum e_col.
__global__ void k_build_T(Geom g, const Entry* ent, const FaceTab* ft, const IfBand* band, const double2* ybuf,
                          size_t ystride, double2* T) {
  const Entry e = ent[blockIdx.x];
  const FaceTab F = ft[e.s];
  const int L = local_if_len(g);
  const double2* x = ybuf + (size_t)blockIdx.x * ystride;
  double2* Ts = T + (size_t)e.s * t_per_sub(g);
  for (int row = threadIdx.x; row < L; row += blockDim.x) {
    int f, ee;
    local_if_face(g, row, &f, &ee);
    double2 v = mk(0.0, 0.0);
    const int io = pick4(F.in_off, f);
    if (io >= 0) {
      const IfBand B = band[io + ee];
      const int len = face_len(g, f), c0 = face_off(g, f);
      for (int d = 0; d < 5; ++d) {
        const int xx = ee + d - 2;
        if (xx >= 0 && xx < len) cfma(v, B.sg[d], x[face_node(g, f, xx)]);
      }
      const int dc = e.rhs - c0 - ee + 1;  // the unit datum's entry relative to ee, shifted by 1
      if (dc >= 0 && dc < 3) v = cadd(v, B.r[dc]);
      v = mk(-v.x, -v.y);
    }
    Ts[t_index(L, row, e.rhs)] = v;
  }
}

constexpr int CG = 64;       // column groups per workgroup (8 rows x 64 groups = 512 threads; 32 and 128 were slower)
constexpr int LMAX = 1024;   // local interface length limit (sub_nx, sub_ny <= 256)

// out[row] = sum_col T[row][col] gin[col] for the rows of one row block; dst[out position] =
// base + sign * out for the rows of the faces in the entry's mask.  Thread (r, grp) takes the
// columns grp + 32 k, so each load instruction of a wavefront reads 8 consecutive columns of the
// block (1 KB contiguous); all its loads are issued before it waits for the incoming data.  The
// column sums meet in a cross-lane tree (lanes r + 8 j) and then across the four wavefronts.
// eft[i] is the face table of entry i's subdomain: the entry, its faces and the row block are
// three independent loads, so the data loads wait for one round trip, not two.
// ALIGNED: every face starts at a multiple of CG, so the CG columns of load k (grp + CG k over the
// workgroup) lie on one face; whether they are needed is then the same in every lane and is
// decided on the scalar unit (loads of faces without data read the block's first columns again).
// KARG: the entry, face table and row block come from the by-value tables sa (small launches),
// read with the kernel arguments, so the operator and data loads follow without another round.
struct NoStepArgs {};
template <typename C, int KMAX, bool ALIGNED, bool KARG>
__global__ __launch_bounds__(kTR * CG) void k_scatter_apply(Geom g, const Entry* ent, const int32_t* rblist,
                                                            const FaceTab* eft, const C* __restrict__ T, SolveIO io,
                                                            std::conditional_t<KARG, StepArgs, NoStepArgs> sa) {
  constexpr int NT = kTR * CG;
  constexpr int GLP = LMAX / NT;  // incoming data per thread
  Entry e;
  FaceTab F;
  int rb;
  if constexpr (KARG) {
    e = sa.e[blockIdx.y];
    F = sa.f[blockIdx.y];
    rb = sa.rb[blockIdx.x];
  } else {
    e = ent[blockIdx.y];
    F = eft[blockIdx.y];
    rb = rblist[blockIdx.x];
  }
  // every table value and kernel argument the workgroup needs is taken into registers here, before
  // the idle-block test below: their scalar loads then go out together instead of one round after
  // the other (the empty statements only name the registers)
  asm volatile("" ::"s"(e.s), "s"(e.rhs), "s"(e.src), "s"(e.mask), "s"(rb));
  asm volatile("" ::"s"(F.in_off[0]), "s"(F.in_off[1]), "s"(F.in_off[2]), "s"(F.in_off[3]));
  asm volatile("" ::"s"(F.out_off[0]), "s"(F.out_off[1]), "s"(F.out_off[2]), "s"(F.out_off[3]));
  asm volatile("" ::"s"(io.g_a), "s"(io.g_b), "s"(io.tr_dst), "s"(io.tr_base), "s"(io.in_faces), "s"(io.copy));
  asm volatile("" ::"s"(T), "s"(g.nif), "s"(io.tr_sign));
  const int L = local_if_len(g);
  const int r = threadIdx.x % kTR, grp = threadIdx.x / kTR;
  // faces present (a neighbour exists: both the incoming and the outgoing block exist)
  const int pm = (F.in_off[0] >= 0) | (F.in_off[1] >= 0) << 1 | (F.in_off[2] >= 0) << 2 | (F.in_off[3] >= 0) << 3;
  const int b1 = g.sny, b2 = 2 * g.sny, b3 = 2 * g.sny + g.snx;  // first rows / columns of faces E, S, N
  // a row block with nothing to write or pass through (only rows of outer or unmasked faces) is
  // skipped whole: the faces it spans are f_lo..f_hi
  {
    const int r0 = rb * kTR, r1 = min(L, r0 + kTR) - 1;
    const int f_lo = (r0 >= b1) + (r0 >= b2) + (r0 >= b3), f_hi = (r1 >= b1) + (r1 >= b2) + (r1 >= b3);
    if ((((e.mask & pm) >> f_lo) & ((2 << (f_hi - f_lo)) - 1)) == 0) return;
  }
  __shared__ double2 gl[LMAX];
  __shared__ double2 red[NT / 64][kTR];
  // 1. incoming data first (absent faces and padding read as zero): every load is issued,
  //    with in-bounds indices, before any is used
  const size_t cb = (size_t)e.rhs * g.nif;
  const int from_b = e.src ? (~io.in_faces & 0xF) : 0;
  // position q of face f sits at in_off[f] + (q - first[f]) of the interface vector
  const int ib0 = F.in_off[0], ib1 = F.in_off[1] - b1, ib2 = F.in_off[2] - b2, ib3 = F.in_off[3] - b3;
  double2 gv[GLP];
  int okm = 0;  // bit k: gv[k] holds data (the others are zeroed when they go to shared memory)
#pragma unroll
  for (int k = 0; k < GLP; ++k) {
    if (ALIGNED && k * NT >= L) {  // no position of this load is on the interface
      gv[k] = mk(0.0, 0.0);
      continue;
    }
    const int q = threadIdx.x + k * NT;
    const bool c1 = q >= b1, c2 = q >= b2, c3 = q >= b3;
    const int f = (int)c1 + (int)c2 + (int)c3;
    int ib = c1 ? ib1 : ib0;  // selects, not branches
    ib = c2 ? ib2 : ib;
    ib = c3 ? ib3 : ib;
    const bool ok = (q < L) & ((pm >> f) & 1);  // bitwise: no branch around the load
    const double2* src = ((from_b >> f) & 1) ? io.g_b : io.g_a;
    gv[k] = src[ok ? cb + ib + q : cb];
    okm |= (int)ok << k;
  }
  // the output row of this thread (threads 0-7): its base value and pass-through datum are
  // loaded up front as well
  const int row = rb * kTR + (int)threadIdx.x;
  int rf, re, oo, io_;
  if constexpr (ALIGNED) {
    // the kTR rows of the block lie on one face: face and block offsets are uniform
    const int r0 = rb * kTR;
    rf = __builtin_amdgcn_readfirstlane((r0 >= b1) + (r0 >= b2) + (r0 >= b3));
    re = row - (rf == 0 ? 0 : rf == 1 ? b1 : rf == 2 ? b2 : b3);
    oo = pick4(F.out_off, rf);
    io_ = pick4(F.in_off, rf);
  } else {
    const int rr = row < L ? row : 0;
    const bool c1 = rr >= b1, c2 = rr >= b2, c3 = rr >= b3;  // selects, not branches
    rf = (int)c1 + (int)c2 + (int)c3;
    int fo = c1 ? b1 : 0, o = c1 ? F.out_off[1] : F.out_off[0], i = c1 ? F.in_off[1] : F.in_off[0];
    fo = c2 ? b2 : fo;
    o = c2 ? F.out_off[2] : o;
    i = c2 ? F.in_off[2] : i;
    fo = c3 ? b3 : fo;
    o = c3 ? F.out_off[3] : o;
    i = c3 ? F.in_off[3] : i;
    re = rr - fo;
    oo = o;
    io_ = i;
  }
  const bool mine = ((int)threadIdx.x < kTR) & (row < L) & ((e.mask >> rf) & 1);
  const bool wr = mine && oo >= 0, cp = mine && io.copy && io_ >= 0;
  double2 bv = mk(0.0, 0.0), cv = mk(0.0, 0.0);
  if (wr && io.tr_base) bv = io.tr_base[cb + oo + re];
  if (cp) cv = io.g_a[cb + io_ + re];
  // 2. the operator rows
  const C* Tb = T + (size_t)e.s * t_per_sub(g) + (size_t)rb * L * kTR + r;
  // columns of absent faces and past L hold no data (their incoming datum is zero): they load the
  // block's column 0 instead, one cached line, so every load stays unconditional
  C v[KMAX];
  if constexpr (ALIGNED) {
    const C* Tl = Tb + (size_t)grp * kTR;
    // bit k: load k reads a face with data (faces span loads [0, b1/CG), [b1/CG, b2/CG), ...)
    auto span = [](int a, int b) -> uint64_t { return ((uint64_t(1) << b) - 1) & ~((uint64_t(1) << a) - 1); };
    const int k1 = b1 / CG, k2 = b2 / CG, k3 = b3 / CG, k4 = L / CG;
    const uint64_t lm64 = ((pm & 1) ? span(0, k1) : 0) | ((pm & 2) ? span(k1, k2) : 0) |
                          ((pm & 4) ? span(k2, k3) : 0) | ((pm & 8) ? span(k3, k4) : 0);
    // read through readfirstlane: a scalar the optimiser cannot see into (it would otherwise merge
    // the redirected loads with the first one and wait for that before issuing the others)
    const uint32_t lm = __builtin_amdgcn_readfirstlane((uint32_t)lm64);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int cc = ((lm >> k) & 1) ? CG * k : 0;  // uniform: a scalar select per load
      v[k] = Tl[(size_t)cc * kTR];
    }
  } else {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int col = grp + CG * k;
      const int f = (col >= b1) + (col >= b2) + (col >= b3);
      const bool live = (col < L) & ((pm >> f) & 1);
      v[k] = Tb[(size_t)(live ? col : 0) * kTR];
    }
  }
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first wait below
#pragma unroll
  for (int k = 0; k < GLP; ++k) gl[threadIdx.x + k * NT] = ((okm >> k) & 1) ? gv[k] : mk(0.0, 0.0);
  __syncthreads();
  double2 acc = mk(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int col = grp + CG * k;
    if (col < L) cfma(acc, to_d(v[k]), gl[col]);
  }
#pragma unroll
  for (int off = kTR; off < 64; off <<= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
  }
  if ((threadIdx.x & 63) < kTR) red[threadIdx.x >> 6][r] = acc;
  __syncthreads();
  if (wr) {
    double2 sum = red[0][r];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) sum = cadd(sum, red[w][r]);
    bv.x += io.tr_sign * sum.x;
    bv.y += io.tr_sign * sum.y;
    io.tr_dst[cb + oo + re] = bv;
  }
  if (cp) io.tr_dst[cb + io_ + re] = cv;
}

}  // namespace

hipError_t launch_build_T(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfBand* band,
                          const double2* ybuf, size_t ystride, double2* T, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_T, dim3(nent), dim3(256), 0, st, g, ent, ft, band, ybuf, ystride, T);
  return hipGetLastError();
}

template <typename C>
hipError_t launch_scatter_apply(const Geom& g, const Entry* ent, int nent, int mask, const int32_t* rblist, int nrb,
                                const FaceTab* eft, const C* T, const SolveIO& io, hipStream_t st, hipEvent_t t0,
                                hipEvent_t t1, const StepArgs* sa) {
  (void)mask;  // carried by every entry
  if (nent == 0 || nrb == 0) return hipSuccess;
  const int L = local_if_len(g);
  if (L > LMAX) return hipErrorInvalidValue;
  if (sa && (nent > kStepArgMax || nrb > kStepArgRb)) return hipErrorInvalidValue;
  const dim3 grid(nrb, nent);
  const bool aligned = g.snx % CG == 0 && g.sny % CG == 0;
  auto go = [&](auto kern, auto tab) {
    // with events, the start and stop times are those of the dispatch itself
    if (t0 || t1)
      hipExtLaunchKernelGGL(kern, grid, dim3(kTR * CG), 0, st, t0, t1, 0, g, ent, rblist, eft, T, io, tab);
    else
      hipLaunchKernelGGL(kern, grid, dim3(kTR * CG), 0, st, g, ent, rblist, eft, T, io, tab);
  };
  auto pick = [&](auto km) {
    constexpr int K = decltype(km)::value;
    if (sa) {
      if (aligned) go(k_scatter_apply<C, K, true, true>, *sa);
      else go(k_scatter_apply<C, K, false, true>, *sa);
    } else {
      if (aligned) go(k_scatter_apply<C, K, true, false>, NoStepArgs{});
      else go(k_scatter_apply<C, K, false, false>, NoStepArgs{});
    }
  };
  if (L <= 8 * CG) pick(std::integral_constant<int, 8>{});
  else if (L <= 16 * CG) pick(std::integral_constant<int, 16>{});
  else pick(std::integral_constant<int, LMAX / CG>{});
  return hipGetLastError();
}

template hipError_t launch_scatter_apply<double2>(const Geom&, const Entry*, int, int, const int32_t*, int,
                                                  const FaceTab*, const double2*, const SolveIO&, hipStream_t,
                                                  hipEvent_t, hipEvent_t, const StepArgs*);
template hipError_t launch_scatter_apply<float2>(const Geom&, const Entry*, int, int, const int32_t*, int,
                                                 const FaceTab*, const float2*, const SolveIO&, hipStream_t, hipEvent_t,
                                                 hipEvent_t, const StepArgs*);
