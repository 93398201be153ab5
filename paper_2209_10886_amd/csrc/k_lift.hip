// Dense lifting operators (paper Sec. 4, eq. (3)): the outgoing data b of the lifting
// w_s = A_s^{-1} f_s with zero transmission data, as one matrix-vector product per subdomain
// with a source, instead of a sequential banded solve on one compute unit.  The same matrices
// give the transmission part of the reconstruction u_s = A_s^{-1} (f_s + B_s g) (Sec. 4).
//
// A_s is complex symmetric (A = A^T), so the row of A_s^{-1} at edge node n(row) equals the
// column A_s^{-1} e_{n(row)} = x_row / inj_row, where x_row = A_s^{-1} B e_row is the unit-datum
// solve already computed for the dense scattering operators.  Stored: W_s[p][row] = x_row[p] /
// inj_row.  Then
//   lifting         y_row = sum_p W_s[p][row] f_s[p] = w_s[n(row)],  b = -Sigma y along each face
//                   (first-order transmission: b_row = -sigma_row y_row);
//   reconstruction  A_s^{-1} B_s g = sum_row x_row g_row = sum_row W_s[.][row] inj_row g_row.
// Layout [s][p][row] (L rows contiguous per node p): a workgroup owns a chunk of nodes and
// accumulates full L-vectors with coalesced loads and no cross-thread reduction; a second pass
// adds the chunk partials in chunk order (deterministic).
#include "hbj_internal.h"

namespace {

constexpr int TE = 32;  // entries (interface positions) per transpose tile
constexpr int TP = 32;  // nodes per transpose tile

// W[s][p][col] = x_e[p] / inj_col for the entries e = (s, col) of a batch.
// Tile of 32 entries x 32 nodes through LDS: coalesced reads along p, writes along col.
__global__ __launch_bounds__(256) void k_build_W(Geom g, const Entry* ent, int nent, const FaceTab* ft,
                                                 const IfCoef* coef, const double2* ybuf, size_t ystride,
                                                 double2* W) {
  __shared__ double2 tile[TE][TP + 1];
  __shared__ double2 scale[TE];
  __shared__ int ss[TE], cc[TE];
  const int e0 = blockIdx.x * TE, p0 = blockIdx.y * TP;
  const int L = local_if_len(g);
  if (threadIdx.x < TE) {
    const int e = e0 + threadIdx.x;
    int s = -1, col = 0;
    double2 sc = mk(0.0, 0.0);
    if (e < nent) {
      const Entry en = ent[e];
      s = en.s;
      col = en.rhs;
      int f, ee;
      local_if_face(g, col, &f, &ee);
      const int io = pick4(ft[s].in_off, f);
      if (io >= 0) {
        sc = cdiv(mk(1.0, 0.0), coef[io + ee].inj);
      }
    }
    ss[threadIdx.x] = s;
    cc[threadIdx.x] = col;
    scale[threadIdx.x] = sc;
  }
  // load: threads along p
  for (int t = threadIdx.x; t < TE * TP; t += blockDim.x) {
    const int j = t / TP, q = t % TP;
    const int e = e0 + j, p = p0 + q;
    tile[j][q] = (e < nent && p < g.nloc) ? ybuf[(size_t)e * ystride + p] : mk(0.0, 0.0);
  }
  __syncthreads();
  // store: threads along the entries (consecutive interface positions of one subdomain)
  for (int t = threadIdx.x; t < TE * TP; t += blockDim.x) {
    const int q = t / TE, j = t % TE;
    const int p = p0 + q, s = ss[j];
    if (s < 0 || p >= g.nloc) continue;
    W[((size_t)s * g.nloc + p) * L + cc[j]] = cmul(scale[j], tile[j][q]);
  }
}

constexpr int RT = 256;

// part[(r * ndom + s) * nchunk + chunk][row] = sum_{p in chunk} W[s][p][row] f_s[p]
// for the (subdomain, rhs) pairs with a nonzero source; a chunk whose source values are all
// exactly zero contributes exactly zero without reading W.
template <int RPT>
__global__ __launch_bounds__(RT) void k_lift_partial(Geom g, const double2* __restrict__ W, const double2* f,
                                                     const int32_t* nz, int pchunk, int nchunk, double2* part) {
  const int chunk = blockIdx.x, s = blockIdx.y, r = blockIdx.z;
  const int ndom = g.n1 * g.n2;
  if (!nz[(size_t)r * ndom + s]) return;
  const int L = local_if_len(g);
  __shared__ double2 fl[1024];
  const int pa = chunk * pchunk, pb = min(g.nloc, pa + pchunk);
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
  const double2* fr = f + (size_t)r * g.nx * g.ny;
  int any = 0;
  for (int p = pa + threadIdx.x; p < pb; p += RT) {
    const int ly = p / g.snx, lx = p - ly * g.snx;
    const double2 v = fr[(size_t)(y0 + ly) * g.nx + x0 + lx];
    fl[p - pa] = v;
    any |= (v.x != 0.0 || v.y != 0.0);
  }
  any = __syncthreads_or(any);
  double2* out = part + ((size_t)(r * ndom + s) * nchunk + chunk) * L;
  double2 acc[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) acc[k] = mk(0.0, 0.0);
  if (any) {
    // batches of 8 nodes: all their loads (clamped, in bounds) are issued before the products
    constexpr int PB = 8;
    const double2* Ws = W + (size_t)s * g.nloc * L;
    for (int p0 = pa; p0 < pb; p0 += PB) {
      double2 wl[PB][RPT];
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int p = min(p0 + i, pb - 1);
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int row = threadIdx.x + k * RT;
          wl[i][k] = Ws[(size_t)p * L + (row < L ? row : L - 1)];
        }
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const double2 fv = (p0 + i < pb) ? fl[p0 + i - pa] : mk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < RPT; ++k) cfma(acc[k], wl[i][k], fv);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int row = threadIdx.x + k * RT;
    if (row < L) out[row] = acc[k];
  }
}

// b[r][out position of row] = -(Sigma y)_row along the row's face, y = the sum of the chunk
// partials (w_s at the edge nodes); zero for subdomains without a source.  Workgroup = 32 output
// rows; y is summed for those rows and two more on each side (Sigma reaches two entries along
// the face) by 8 chunk groups: group k adds chunks k, k + 8, ... in order, then the 8 group sums
// are added in group order (a fixed order: the result is deterministic).
constexpr int kLiftHalo = 2;
__global__ __launch_bounds__(RT) void k_lift_reduce(Geom g, const FaceTab* ft, const IfBand* band, const int32_t* nz,
                                                    const double2* part, int nchunk, double2* b) {
  constexpr int NY = 32 + 2 * kLiftHalo;
  const int s = blockIdx.y, r = blockIdx.z;
  const int ndom = g.n1 * g.n2;
  const int L = local_if_len(g);
  const int lr = threadIdx.x % 32, k = threadIdx.x / 32;
  const int r0 = blockIdx.x * 32 - kLiftHalo;  // first row of the y window
  const bool has = nz[(size_t)r * ndom + s] != 0;
  __shared__ double2 red[8][NY];
  __shared__ double2 y[NY];
  for (int w = lr; w < NY; w += 32) {
    const int row = r0 + w;
    double2 acc = mk(0.0, 0.0);
    if (has && row >= 0 && row < L) {
      const double2* ps = part + (size_t)(r * ndom + s) * nchunk * L + row;
      for (int c = k; c < nchunk; c += 8) acc = cadd(acc, ps[(size_t)c * L]);
    }
    red[k][w] = acc;
  }
  __syncthreads();
  if (k == 0) {
    for (int w = lr; w < NY; w += 32) {
      double2 t = red[0][w];
      for (int q = 1; q < 8; ++q) t = cadd(t, red[q][w]);
      y[w] = t;
    }
  }
  __syncthreads();
  const int row = blockIdx.x * 32 + lr;
  if (k == 0 && row < L) {
    int f, e;
    local_if_face(g, row, &f, &e);
    const FaceTab F = ft[s];
    const int oo = pick4(F.out_off, f), io = pick4(F.in_off, f);
    if (oo >= 0) {
      const IfBand B = band[io + e];
      const int len = face_len(g, f);
      double2 t = mk(0.0, 0.0);
      for (int d = 0; d < 5; ++d) {
        const int xx = e + d - 2;  // entry along the face; its row is row + d - 2
        if (xx >= 0 && xx < len) cfma(t, B.sg[d], y[lr + d]);
      }
      b[(size_t)r * g.nif + oo + e] = mk(-t.x, -t.y);
    }
  }
}

// u_s[p] = (nz ? u_s[p] : 0) + sum_row W_s[p][row] gs_row with gs_row = inj_row * g_row
// (the incoming datum of the row's face; 0 on outer faces).  u_s already holds A_s^{-1} f_s for
// the subdomains with a source.  A wavefront per node p reads its 8 KB row of W coalesced
// (KL entries per lane) and reduces across lanes; each wavefront takes 8 nodes, 32 / KL at a time.
constexpr int kReconPW = 8;  // nodes per wavefront of the dense reconstruction (16 and 32: the same time)
template <int KL>
__global__ __launch_bounds__(RT) void k_recon_dense(Geom g, const FaceTab* ft, const IfCoef* coef,
                                                    const double2* __restrict__ W, const double2* gin,
                                                    const int32_t* nz, double2* u) {
  constexpr int PW = kReconPW, PB = 32 / KL;  // nodes per wavefront, nodes in flight
  const int s = blockIdx.y, r = blockIdx.z;
  const int ndom = g.n1 * g.n2;
  const int L = local_if_len(g);
  const FaceTab F = ft[s];
  __shared__ double2 gs[KL * 64];
  for (int col = threadIdx.x; col < KL * 64; col += RT) {
    double2 v = mk(0.0, 0.0);
    if (col < L) {
      int f, e;
      local_if_face(g, col, &f, &e);
      const int io = pick4(F.in_off, f);
      if (io >= 0) {
        v = cmul(coef[io + e].inj, gin[(size_t)r * g.nif + io + e]);
      }
    }
    gs[col] = v;
  }
  __syncthreads();
  const bool has = nz[(size_t)r * ndom + s] != 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x0 = (s % g.n1) * g.snx, y0 = (s / g.n1) * g.sny;
  const double2* Ws = W + (size_t)s * g.nloc * L;
  // columns of faces on the outer boundary carry no trace (gs = 0 there): their loads are
  // redirected to column 0 of the same node, a line the wavefront reads anyway, so those
  // matrix entries cost no memory traffic
  int cidx[KL];
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const int col = lane + 64 * k;
    int f = 0, e = 0;
    if (col < L) local_if_face(g, col, &f, &e);
    cidx[k] = (col < L && pick4(F.in_off, f) >= 0) ? col : 0;
  }
  double2* ur = u + (size_t)r * g.nx * g.ny;
  const int pbase = blockIdx.x * (RT / 64) * PW + wv * PW;
  for (int i0 = 0; i0 < PW; i0 += PB) {
    double2 wl[PB][KL];
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int p = min(pbase + i0 + i, g.nloc - 1);
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        wl[i][k] = Ws[(size_t)p * L + cidx[k]];
      }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      double2 acc = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < KL; ++k) cfma(acc, wl[i][k], gs[lane + 64 * k]);  // gs is 0 past L
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off);
        acc.y += __shfl_xor(acc.y, off);
      }
      const int p = pbase + i0 + i;
      if (lane == 0 && p < g.nloc) {
        const int ly = p / g.snx, lx = p - ly * g.snx;
        const size_t o = (size_t)(y0 + ly) * g.nx + x0 + lx;
        double2 b = has ? ur[o] : mk(0.0, 0.0);
        ur[o] = cadd(b, acc);
      }
    }
  }
}

}  // namespace

hipError_t launch_recon_dense(const Geom& g, const FaceTab* ft, const IfCoef* coef, const double2* W,
                              const double2* gin, const int32_t* nz, int nrhs, double2* u, hipStream_t st) {
  const int L = local_if_len(g);
  if (L > 1024) return hipErrorInvalidValue;
  constexpr int nodes = (RT / 64) * kReconPW;  // per workgroup
  const dim3 grid((g.nloc + nodes - 1) / nodes, g.n1 * g.n2, nrhs);
  if (L <= 512) hipLaunchKernelGGL((k_recon_dense<8>), grid, dim3(RT), 0, st, g, ft, coef, W, gin, nz, u);
  else hipLaunchKernelGGL((k_recon_dense<16>), grid, dim3(RT), 0, st, g, ft, coef, W, gin, nz, u);
  return hipGetLastError();
}

hipError_t launch_build_W(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfCoef* coef,
                          const double2* ybuf, size_t ystride, double2* W, hipStream_t st) {
  if (nent == 0) return hipSuccess;
  const dim3 grid((nent + TE - 1) / TE, (g.nloc + TP - 1) / TP);
  hipLaunchKernelGGL(k_build_W, grid, dim3(256), 0, st, g, ent, nent, ft, coef, ybuf, ystride, W);
  return hipGetLastError();
}

int lift_chunks(const Geom& g, int pchunk) { return (g.nloc + pchunk - 1) / pchunk; }

hipError_t launch_lift_partials(const Geom& g, const double2* W, const double2* f, const int32_t* nz, int nrhs,
                                int pchunk, double2* part, hipStream_t st) {
  const int L = local_if_len(g);
  if (pchunk > 1024 || L > 1024) return hipErrorInvalidValue;
  const int nchunk = lift_chunks(g, pchunk);
  const dim3 grid(nchunk, g.n1 * g.n2, nrhs);
  if (L <= RT) hipLaunchKernelGGL((k_lift_partial<1>), grid, dim3(RT), 0, st, g, W, f, nz, pchunk, nchunk, part);
  else if (L <= 2 * RT)
    hipLaunchKernelGGL((k_lift_partial<2>), grid, dim3(RT), 0, st, g, W, f, nz, pchunk, nchunk, part);
  else hipLaunchKernelGGL((k_lift_partial<4>), grid, dim3(RT), 0, st, g, W, f, nz, pchunk, nchunk, part);
  return hipGetLastError();
}

hipError_t launch_lift_dense(const Geom& g, const FaceTab* ft, const IfBand* band, const double2* W, const double2* f,
                             const int32_t* nz, int nrhs, int pchunk, double2* part, double2* b, hipStream_t st) {
  const int L = local_if_len(g);
  const int nchunk = lift_chunks(g, pchunk);
  hipError_t e = launch_lift_partials(g, W, f, nz, nrhs, pchunk, part, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lift_reduce, dim3((L + 31) / 32, g.n1 * g.n2, nrhs), dim3(RT), 0, st, g, ft, band, nz, part,
                     nchunk, b);
  return hipGetLastError();
}
