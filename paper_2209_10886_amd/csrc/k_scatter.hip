// Dense local scattering operators (paper Sec. 4, the operators S_{m(j,i), m(i,k)}).
//
// For subdomain s the map from its incoming Robin data (all faces, local interface
// order W, E, S, N) to its outgoing data is linear:
//   out = T_s g,   T_s = -diag(rho) - diag(sigma) R A_s^{-1} B
// with B the injection g / (beta- h^2) on the edge rows and R the restriction to the
// edge nodes.  Column c of T_s is built from one local solve with a unit datum at
// position c.  Applying T_s is then a dense matrix-vector product whose rows can be
// spread over many workgroups, instead of one workgroup walking the whole band.
#include "hbj_internal.h"

namespace {

// T[s][col][row] for every entry (s, col): x = A_s^{-1} B e_col is in ybuf[entry]
__global__ void k_build_T(Geom g, const Entry* ent, const FaceTab* ft, const IfCoef* coef, const double2* ybuf,
                          size_t ystride, double2* T) {
  const Entry e = ent[blockIdx.x];
  const FaceTab F = ft[e.s];
  const int L = local_if_len(g);
  const double2* x = ybuf + (size_t)blockIdx.x * ystride;
  double2* col = T + ((size_t)e.s * L + e.rhs) * L;
  for (int row = threadIdx.x; row < L; row += blockDim.x) {
    int f, ee;
    local_if_face(g, row, &f, &ee);
    double2 v = mk(0.0, 0.0);
    if (F.in_off[f] >= 0) {
      const IfCoef c = coef[F.in_off[f] + ee];
      v = cmul(c.sigma, x[face_node(g, f, ee)]);
      v = mk(-v.x, -v.y);
      if (row == e.rhs) {
        v.x -= c.rho.x;
        v.y -= c.rho.y;
      }
    }
    col[row] = v;
  }
}

constexpr int RT = 32;       // rows per workgroup
constexpr int CGROUPS = 8;   // column groups (two per face)
constexpr int LMAX = 1024;   // local interface length limit (sub_nx, sub_ny <= 256)

// out[row] = sum_col T[col][row] gin[col] for the rows of the faces in the entry's mask;
// dst[out position] = base + sign * out.  One workgroup per (32-row tile, entry).
template <typename C>
__global__ __launch_bounds__(RT * CGROUPS) void k_scatter_apply(Geom g, const Entry* ent, const FaceTab* ft,
                                                                const C* __restrict__ T, SolveIO io) {
  const Entry e = ent[blockIdx.y];
  const FaceTab F = ft[e.s];
  const int L = local_if_len(g);
  const int row = blockIdx.x * RT + (threadIdx.x % RT);
  const int grp = threadIdx.x / RT;
  int rf = 0, re = 0;
  bool active = row < L;
  if (active) {
    local_if_face(g, row, &rf, &re);
    active = ((e.mask >> rf) & 1) && F.out_off[rf] >= 0;
  }
  if (!__syncthreads_or(active)) return;
  __shared__ double2 gl[LMAX];
  __shared__ double2 red[CGROUPS][RT];
  const double2* gin = e.src ? io.g_b : io.g_a;
  gin += (size_t)e.rhs * g.nif;
  for (int q = threadIdx.x; q < L; q += blockDim.x) {
    int f, ee;
    local_if_face(g, q, &f, &ee);
    gl[q] = (F.in_off[f] >= 0) ? gin[F.in_off[f] + ee] : mk(0.0, 0.0);
  }
  __syncthreads();
  // column group -> half of one face
  const int cf = grp >> 1, half = grp & 1;
  double2 acc = mk(0.0, 0.0);
  if (F.in_off[cf] >= 0 && row < L) {
    const int len = face_len(g, cf), off = face_off(g, cf);
    const int c0 = off + (half ? len / 2 : 0), c1 = off + (half ? len : len / 2);
    const C* Tc = T + (size_t)e.s * L * L + row;
#pragma unroll 4
    for (int c = c0; c < c1; ++c) cfma(acc, to_d(Tc[(size_t)c * L]), gl[c]);
  }
  red[grp][threadIdx.x % RT] = acc;
  __syncthreads();
  if (grp == 0 && active) {
    double2 s = red[0][threadIdx.x];
#pragma unroll
    for (int k = 1; k < CGROUPS; ++k) s = cadd(s, red[k][threadIdx.x]);
    const size_t o = (size_t)e.rhs * g.nif + F.out_off[rf] + re;
    double2 base = io.tr_base ? io.tr_base[o] : mk(0.0, 0.0);
    base.x += io.tr_sign * s.x;
    base.y += io.tr_sign * s.y;
    io.tr_dst[o] = base;
  }
}

}  // namespace

hipError_t launch_build_T(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfCoef* coef,
                          const double2* ybuf, size_t ystride, double2* T, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_T, dim3(nent), dim3(256), 0, st, g, ent, ft, coef, ybuf, ystride, T);
  return hipGetLastError();
}

template <typename C>
hipError_t launch_scatter_apply(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const C* T,
                                const SolveIO& io, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  const int L = local_if_len(g);
  if (L > LMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_scatter_apply<C>), dim3((L + RT - 1) / RT, nent), dim3(RT * CGROUPS), 0, st, g, ent, ft, T,
                     io);
  return hipGetLastError();
}

template hipError_t launch_scatter_apply<double2>(const Geom&, const Entry*, int, const FaceTab*, const double2*,
                                                  const SolveIO&, hipStream_t);
template hipError_t launch_scatter_apply<float2>(const Geom&, const Entry*, int, const FaceTab*, const float2*,
                                                 const SolveIO&, hipStream_t);
