// Dense local scattering operators (paper Sec. 4, the operators S_{m(j,i), m(i,k)}).
// Storage: T[s][col][row], column-major, L x L per subdomain.
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

// T[s][col][row] (column-major) for every entry (s, col): x = A_s^{-1} B e_col is in ybuf[entry]
__global__ void k_build_T(Geom g, const Entry* ent, const FaceTab* ft, const IfCoef* coef, const double2* ybuf,
                          size_t ystride, double2* T) {
  const Entry e = ent[blockIdx.x];
  const FaceTab F = ft[e.s];
  const int L = local_if_len(g);
  const double2* x = ybuf + (size_t)blockIdx.x * ystride;
  double2* Ts = T + (size_t)e.s * L * L;
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
    Ts[(size_t)e.rhs * L + row] = v;
  }
}

constexpr int ROWS = 8;      // output rows per workgroup
constexpr int CG = 32;       // column groups per workgroup (256 threads)
constexpr int LMAX = 1024;   // local interface length limit (sub_nx, sub_ny <= 256)

// Row r of the concatenation of the faces selected by mask (W, E, S, N order).
__device__ inline int masked_row(const Geom& g, int mask, int r) {
  for (int f = 0; f < 4; ++f) {
    if (!((mask >> f) & 1)) continue;
    const int len = face_len(g, f);
    if (r < len) return face_off(g, f) + r;
    r -= len;
  }
  return -1;
}

// out[row] = sum_col T[col][row] gin[col] for the rows of the faces in the entry's mask;
// dst[out position] = base + sign * out.  Workgroup = 8 rows x 32 column groups over the
// masked rows only; each thread issues all its column loads (8 consecutive rows = 128 B per
// column) before it waits for the incoming data, then the 32 partial sums meet in LDS.
template <typename C, int KMAX>
__global__ __launch_bounds__(ROWS * CG) void k_scatter_apply(Geom g, const Entry* ent, const FaceTab* ft,
                                                             const C* __restrict__ T, SolveIO io) {
  const Entry e = ent[blockIdx.y];
  const int L = local_if_len(g);
  const int r = threadIdx.x % ROWS, grp = threadIdx.x / ROWS;
  const int row = masked_row(g, e.mask, blockIdx.x * ROWS + r);
  const int nk = (L + CG - 1) / CG, c0 = grp * nk;
  const C* Tc = T + (size_t)e.s * L * L + (row < 0 ? 0 : row);
  C v[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    v[k].x = 0;
    v[k].y = 0;
    if (k < nk && row >= 0 && c0 + k < L) v[k] = Tc[(size_t)(c0 + k) * L];
  }
  const FaceTab F = ft[e.s];
  __shared__ double2 gl[LMAX];
  __shared__ double2 red[CG][ROWS + 1];
  const double2* gin = (e.src ? io.g_b : io.g_a) + (size_t)e.rhs * g.nif;
  for (int f = 0; f < 4; ++f) {  // absent faces read as zero data
    const int off = face_off(g, f), len = face_len(g, f);
    for (int q = threadIdx.x; q < len; q += blockDim.x)
      gl[off + q] = (F.in_off[f] >= 0) ? gin[F.in_off[f] + q] : mk(0.0, 0.0);
  }
  __syncthreads();
  double2 acc = mk(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < nk && c0 + k < L) cfma(acc, to_d(v[k]), gl[c0 + k]);
  red[grp][r] = acc;
  __syncthreads();
  if (threadIdx.x < ROWS && row >= 0) {
    int rf, re;
    local_if_face(g, row, &rf, &re);
    if (F.out_off[rf] >= 0) {
      double2 sum = red[0][r];
#pragma unroll 8
      for (int k = 1; k < CG; ++k) sum = cadd(sum, red[k][r]);
      const size_t o = (size_t)e.rhs * g.nif + F.out_off[rf] + re;
      double2 base = io.tr_base ? io.tr_base[o] : mk(0.0, 0.0);
      base.x += io.tr_sign * sum.x;
      base.y += io.tr_sign * sum.y;
      io.tr_dst[o] = base;
    }
  }
}

// Full operator (every face of every subdomain): long streams per thread.  Workgroup =
// 32 rows x 8 column groups; each column read by a wavefront is 32 consecutive rows (512 B).
template <typename C>
__global__ __launch_bounds__(256) void k_scatter_full(Geom g, const Entry* ent, const FaceTab* ft,
                                                      const C* __restrict__ T, SolveIO io) {
  constexpr int R32 = 32, G8 = 8;
  const Entry e = ent[blockIdx.y];
  const FaceTab F = ft[e.s];
  const int L = local_if_len(g);
  const int row = blockIdx.x * R32 + (threadIdx.x % R32);
  const int grp = threadIdx.x / R32;
  __shared__ double2 gl[LMAX];
  __shared__ double2 red[G8][R32 + 1];
  const double2* gin = (e.src ? io.g_b : io.g_a) + (size_t)e.rhs * g.nif;
  for (int f = 0; f < 4; ++f) {
    const int off = face_off(g, f), len = face_len(g, f);
    for (int q = threadIdx.x; q < len; q += blockDim.x)
      gl[off + q] = (F.in_off[f] >= 0) ? gin[F.in_off[f] + q] : mk(0.0, 0.0);
  }
  __syncthreads();
  double2 acc = mk(0.0, 0.0);
  if (row < L) {
    const int nk = (L + G8 - 1) / G8, c0 = grp * nk, c1 = min(L, c0 + nk);
    const C* Tc = T + (size_t)e.s * L * L + row;
#pragma unroll 8
    for (int c = c0; c < c1; ++c) cfma(acc, to_d(Tc[(size_t)c * L]), gl[c]);
  }
  red[grp][threadIdx.x % R32] = acc;
  __syncthreads();
  if (threadIdx.x < R32 && row < L) {
    int rf, re;
    local_if_face(g, row, &rf, &re);
    if (((e.mask >> rf) & 1) && F.out_off[rf] >= 0) {
      double2 sum = red[0][threadIdx.x];
#pragma unroll
      for (int k = 1; k < G8; ++k) sum = cadd(sum, red[k][threadIdx.x]);
      const size_t o = (size_t)e.rhs * g.nif + F.out_off[rf] + re;
      double2 base = io.tr_base ? io.tr_base[o] : mk(0.0, 0.0);
      base.x += io.tr_sign * sum.x;
      base.y += io.tr_sign * sum.y;
      io.tr_dst[o] = base;
    }
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
hipError_t launch_scatter_apply(const Geom& g, const Entry* ent, int nent, int mask, const FaceTab* ft, const C* T,
                                const SolveIO& io, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  const int L = local_if_len(g);
  if (L > LMAX) return hipErrorInvalidValue;
  int rows = 0;
  for (int f = 0; f < 4; ++f)
    if ((mask >> f) & 1) rows += face_len(g, f);
  if (mask == 0xF) {
    hipLaunchKernelGGL((k_scatter_full<C>), dim3((L + 31) / 32, nent), dim3(256), 0, st, g, ent, ft, T, io);
    return hipGetLastError();
  }
  const dim3 grid((rows + ROWS - 1) / ROWS, nent);
  if (L <= 16 * CG) hipLaunchKernelGGL((k_scatter_apply<C, 16>), grid, dim3(ROWS * CG), 0, st, g, ent, ft, T, io);
  else hipLaunchKernelGGL((k_scatter_apply<C, LMAX / CG>), grid, dim3(ROWS * CG), 0, st, g, ent, ft, T, io);
  return hipGetLastError();
}

template hipError_t launch_scatter_apply<double2>(const Geom&, const Entry*, int, int, const FaceTab*,
                                                  const double2*, const SolveIO&, hipStream_t);
template hipError_t launch_scatter_apply<float2>(const Geom&, const Entry*, int, int, const FaceTab*, const float2*,
                                                 const SolveIO&, hipStream_t);
