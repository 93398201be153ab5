// Internal declarations shared by the HIP kernels and the host runtime of libhbj.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/hbj.h"

// ---------------------------------------------------------------------------
// complex arithmetic on HIP vector types (x = real, y = imaginary)
// ---------------------------------------------------------------------------
template <typename R> struct Cplx;
template <> struct Cplx<double> { typedef double2 T; };
template <> struct Cplx<float> { typedef float2 T; };

__host__ __device__ inline double2 mk(double a, double b) { return make_double2(a, b); }
__host__ __device__ inline float2 mkf(float a, float b) { return make_float2(a, b); }

template <typename V> __host__ __device__ inline V cadd(V a, V b) { a.x += b.x; a.y += b.y; return a; }
template <typename V> __host__ __device__ inline V csub(V a, V b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename V> __host__ __device__ inline V cmul(V a, V b) {
  V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename V> __host__ __device__ inline V cconj(V a) { a.y = -a.y; return a; }
// acc += a * b
template <typename V> __host__ __device__ inline void cfma(V& acc, V a, V b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename V> __host__ __device__ inline void cfma_conj(V& acc, V a, V b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  double r = b.x / b.y, d = b.y + b.x * r;
  return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__host__ __device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

template <typename V> __device__ inline V to_c(double2 a);
template <> __device__ inline double2 to_c<double2>(double2 a) { return a; }
template <> __device__ inline float2 to_c<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
__device__ inline double2 to_d(double2 a) { return a; }
__device__ inline double2 to_d(float2 a) { return make_double2((double)a.x, (double)a.y); }

// ---------------------------------------------------------------------------
// problem geometry as seen by the kernels
// ---------------------------------------------------------------------------
enum { FACE_W = 0, FACE_E = 1, FACE_S = 2, FACE_N = 3 };

struct Geom {
  int nx, ny;        // global interior grid
  int n1, n2;        // checkerboard
  int snx, sny;      // subdomain size
  int nloc;          // snx * sny
  int kl, ku, kv;    // band: kl = ku = snx, kv = kl + ku
  int ldab;          // 2 kl + ku + 1
  int nif;           // interface length
  double h, k;
};

// solve layout of the blocked triangular solves
struct SolveLayout {
  int nb;            // block (panel) width
  int nblk;          // ceil(nloc / nb)
  int wf;            // forward window rows  = nb + kl
  int wb;            // backward window rows = nb + kvb: kvb = kv = kl + ku (the band of U with row
                     // interchanges), or ku when no subdomain's factorisation interchanged rows
  int cgf, cgb;      // lanes sharing one window row (column groups) in the forward / backward kernels
  size_t mf_per_sub; // entries of the forward M per subdomain  = nblk * nb * wf
  size_t mb_per_sub; // entries of the backward M per subdomain = nblk * nb * wb
  size_t pf_per_sub; // int16 permutation entries per subdomain  = nblk * wf
};

// rows of U above a column block that the backward solves carry (kv or ku, see wb)
__host__ __device__ inline int solve_kvb(const SolveLayout& L) { return L.wb - L.nb; }

// Position of entry (column c, window row r) of one block's solve matrix in the
// thread-tiled layout [k][r][cg] with c = cg * (nb / cg) + k: lane (r, cg) of the solve
// kernel reads its k-th value at ((k * rows + r) * cg_count + cg), so every load
// instruction of a wavefront is one contiguous run.
__host__ __device__ inline size_t tile_index(int c, int r, int rows, int nb, int cg) {
  const int nc = nb / cg;
  return ((size_t)(c % nc) * rows + r) * cg + c / nc;
}

// one local solve of a batched launch
struct Entry {
  int32_t s;      // subdomain index (i2-1)*n1 + (i1-1)
  int32_t rhs;    // right-hand-side column
  int32_t src;    // 0: incoming data from g_a, 1: from g_b
  int32_t mask;   // bit f set: write the outgoing trace of face f
};

// per-subdomain face table: offsets into the interface vector (-1 = outer face)
struct FaceTab {
  int32_t in_off[4];   // block m(i, j): data received by i through face f
  int32_t out_off[4];  // block m(j, i): data sent by i through face f
};

// interface coefficients of every interface position (same on both sides of a face); alpha
// here is the impedance of the transmission condition (alpha a for the second-order one)
struct IfCoef {
  double2 rho;    // beta+ / beta-
  double2 sigma;  // 2 i alpha / (h beta-)
  double2 inj;    // 1 / (beta- h^2)
};

// Face-line maps of the transmission condition at interface position q (entry e of its face):
// the datum sent across the face at e is -sum_d r[d] g_{e+d-1} - sum_d sg[d] u_{e+d-2} over the
// entries of the same face (r = R, sg = Sigma; first order: r = (0, rho, 0), sg = (0, 0, sigma,
// 0, 0)), and t[0], t[1] are the tangential edge weights s_{e-1,e}, s_{e,e+1} of the second-order
// condition (the row of the edge node gains -(C u)_e / h^2, C the tangential operator; zero for
// the first-order condition).
struct IfBand {
  double2 r[3];
  double2 sg[5];
  double2 t[2];
};

// How a local-solve launch obtains its right-hand side and where results go.
struct SolveIO {
  // right-hand side: (f restricted) + injected Robin data, or an explicit buffer
  const double2* f;       // [nrhs][ny][nx] or null
  const double2* g_a;     // incoming data, [nrhs][nif] or null
  const double2* g_b;     // second source (entries with src = 1)
  const double2* rhs64;   // explicit local right-hand sides [entry][nloc] (overrides f/g)
  // outputs
  double2* u;             // global field [nrhs][ny][nx] or null
  double2* x64;           // local solutions [entry][nloc] (complex128) or null
  double2* tr_dst;        // trace destination [nrhs][nif] or null
  const double2* tr_base; // dst = base + sign * out ; null = 0
  double tr_sign;
  int tr_reflect;         // include -rho g (the incoming data) in the outgoing trace
  int unit;               // right-hand side = unit Robin datum at local interface position entry.rhs
  const int32_t* nz;      // [nrhs][ndom] 0 = the entry's source restriction is identically zero and
                          // the entry has no incoming data: its solution is 0 (the solve is skipped)
  // dense operators only: faces always read from g_a (also for entries with src = 1), and
  // copy = 1 writes tr_dst = g_a on the entry's own incoming positions of the faces in its
  // mask (a pass then needs no pre-filled output)
  int in_faces;
  int copy;
  // with nz: entries without a source write nothing at all (their field is rebuilt elsewhere)
  int nz_skip_out;
  // dense operators on the matrix-product path only: dst = base - sub + sign * out (null = 0)
  const double2* tr_sub;
  // sweep steps on the matrix-product path, chained: the output at interface position p is also
  // stored, in the element type of the products, at ctile[cmap[p] * crpad + rhs] when cmap[p] >= 0
  // (the gathered tile of the next step)
  const int32_t* cmap;
  void* ctile;
  int crpad;
};

// Local interface positions of a subdomain: faces W, E, S, N in this order, each with
// its entries ordered along the face; L = 2 sny + 2 snx.
__host__ __device__ inline int face_len(const Geom& g, int f) { return f < 2 ? g.sny : g.snx; }
__host__ __device__ inline int face_off(const Geom& g, int f) {
  return f == 0 ? 0 : f == 1 ? g.sny : f == 2 ? 2 * g.sny : 2 * g.sny + g.snx;
}
__host__ __device__ inline int local_if_len(const Geom& g) { return 2 * g.sny + 2 * g.snx; }
__host__ __device__ inline void local_if_face(const Geom& g, int q, int* f, int* ee) {
  int ff = (q < g.sny) ? 0 : (q < 2 * g.sny) ? 1 : (q < 2 * g.sny + g.snx) ? 2 : 3;
  *f = ff;
  *ee = q - face_off(g, ff);
}
// local row of the edge node of face f, entry ee
__host__ __device__ inline int face_node(const Geom& g, int f, int ee) {
  return f == 0 ? ee * g.snx : f == 1 ? ee * g.snx + g.snx - 1 : f == 2 ? ee : (g.sny - 1) * g.snx + ee;
}

// Dense scattering operators T_s (L x L): blocks of kTR rows, T[s][row / kTR][col][row % kTR],
// the row count padded to a multiple of kTR (padding rows are zero).  A workgroup that owns a
// row block streams one contiguous run of kTR * L entries.
constexpr int kTR = 8;
__host__ __device__ inline int t_rows(const Geom& g) { return (local_if_len(g) + kTR - 1) / kTR * kTR; }
__host__ __device__ inline size_t t_per_sub(const Geom& g) { return (size_t)t_rows(g) * local_if_len(g); }
__host__ __device__ inline size_t t_index(int L, int row, int col) {
  return ((size_t)(row / kTR) * L + col) * kTR + (row % kTR);
}
// Tables of a small stepped launch of the dense operators, passed by value: a workgroup then has
// its entry, face table and row block with its kernel arguments, and its operator loads need no
// dependent table load first.
constexpr int kStepArgMax = 16;   // entries
constexpr int kStepArgRb = 128;   // row blocks (local interface length <= 1024)
struct StepArgs {
  Entry e[kStepArgMax];
  FaceTab f[kStepArgMax];  // face table of entry i's subdomain
  int32_t rb[kStepArgRb];  // the launch's row blocks
};
__host__ __device__ inline int pick4(const int32_t (&a)[4], int f) {
  return f == 0 ? a[0] : f == 1 ? a[1] : f == 2 ? a[2] : a[3];
}

// Dataflow sweeps: every sweep step of a preconditioner application (and the operator that
// follows it) in one launch.  A task is one row block of one (stage, subdomain, right-hand
// side); workgroups claim tasks in a fixed topological order from a ticket counter and wait
// only on tasks of smaller tickets, through per-(stage, subdomain, rhs) completion counters.
constexpr int kDfMaxDeps = 5;
constexpr int kDfMaxStages = 3;
struct DfTask {
  int32_t stage, s, rhs, rb;
  int32_t first;             // 1: every face is read from the stage input (first step of an interval)
  int32_t slot;              // completion counter incremented when the task is done
  int32_t ndep;
  int32_t dep[kDfMaxDeps];   // counters waited for
  int32_t need[kDfMaxDeps];  // value each must reach (the number of tasks behind it)
  int32_t pad;
};
// One stage: dst[o] = base[o] + sign (T_s g_s)[row] for the rows of the faces in `mask`,
// g_s read from `out` on the faces in `out_read` (after the first step) and from `in` elsewhere;
// with `copy`, dst = in on the subdomain's own incoming positions of the faces in `mask`
// (positions no task of the stage writes).
struct DfStage {
  const double2* in;
  const double2* out;
  double2* dst;
  const double2* base;
  double sign;
  int32_t mask, out_read, copy, pad;
};
struct DfArgs {
  DfStage st[kDfMaxStages];
};

// ---------------------------------------------------------------------------
// launchers (each returns hipError_t of the launch)
// ---------------------------------------------------------------------------
hipError_t launch_check_medium(const double* c, int n, int* bad, hipStream_t st);
hipError_t launch_c_to_m(const double* c, double* m, int n, hipStream_t st);
// ta, tb: the (a, b) of the transmission condition d_n u - i alpha a u - (i b / alpha) d_tt u = g
// ((1, 0) for the first-order condition)
hipError_t launch_if_coef(const Geom& g, const double* m, const int32_t* pos_tab, double2 ta, IfCoef* coef,
                          hipStream_t st);
hipError_t launch_if_band(const Geom& g, const double* m, const int32_t* pos_tab, int order, double2 ta, double2 tb,
                          const IfCoef* coef, IfBand* band, hipStream_t st);
hipError_t launch_local_diag(const Geom& g, const double* m, const FaceTab* ft, const IfCoef* coef, const IfBand* band,
                             double2* diag, hipStream_t st);
hipError_t launch_band_assemble(const Geom& g, const double2* diag, const FaceTab* ft, const IfBand* band, double2* ab,
                                int nsub, hipStream_t st);
// blocked: panels of 16 columns (the same factors; falls back to the column-by-column kernel when the
// panel does not fit in LDS)
hipError_t launch_band_lu(const Geom& g, double2* ab, int32_t* ipiv, int32_t* info, int nsub, hipStream_t st,
                          bool blocked = true);
hipError_t launch_repack(const Geom& g, const SolveLayout& L, const double2* ab, const int32_t* ipiv,
                         double2* mf, int16_t* pf, int32_t* pflag, double2* mb, int nsub, hipStream_t st);
hipError_t launch_cast_c64(const double2* src, float2* dst, size_t n, hipStream_t st);

void solve_column_groups(int wf, int wb, int* cgf, int* cgb);
// Process-wide cache of autotuned choices, persisted as a JSON file (tune_cache.cpp).
bool tune_cache_get(const std::string& key, int* variant);
bool tune_cache_put(const std::string& key, int variant, const float* us, int n);

// One workgroup per (subdomain, right-hand side).  dv selects the register prefetch depth
// (0: default; 1, 2: the alternatives the autotuner times); every depth gives the same result.
constexpr int kSolveDepthVariants = 3;
int solve_depth(bool fwd, size_t real_bytes, int dv);
template <typename R>
hipError_t launch_fwd(const Geom& g, const SolveLayout& L, const Entry* ent, int nent, const FaceTab* ft,
                      const IfCoef* coef, const typename Cplx<R>::T* mf, const int16_t* pf, const int32_t* pflag,
                      const SolveIO& io,
                      typename Cplx<R>::T* ybuf, hipStream_t st, int dv = 0);
template <typename R>
hipError_t launch_bwd(const Geom& g, const SolveLayout& L, const Entry* ent, int nent, const FaceTab* ft,
                      const IfCoef* coef, const typename Cplx<R>::T* mb, const SolveIO& io,
                      typename Cplx<R>::T* ybuf, hipStream_t st, int dv = 0);

// The same solves with each local solve split over np workgroups (a run of bpp column blocks
// each): two passes over the runs and, between them, a chain over the runs' transfer matrices
// (formed by launch_part_phi once per factorisation); results as launch_fwd / launch_bwd up to
// rounding.  rb: the solve buffer (the right-hand sides, then the solutions, as launch_fwd and
// launch_bwd leave them); y2: the forward results, [entry][nblk nb]; sig, tt: [entry][np][ns]
// states; phi_f [subdomain][np - 2][kl][kl], phi_b [subdomain][np - 2][kv][kv]; pw: the chain's
// counters.
struct PartLayout {
  int np;   // runs per solve (>= 2), each nonempty
  int bpp;  // column blocks per run (the last run may be shorter)
  int ns;   // state stride of sig / tt (>= kv)
};
// ticket counters of the chain launches: two regions of part_chain_counters(entries, np) (one
// per entry), used by alternate launches (parity, toggled by each launch), each launch zeroing
// the other region; a failed wait sets *err
struct PartWait {
  int32_t* ctr;
  int nctr;
  int parity;
  int32_t* err;
  int spin;
};
constexpr int kChainGridMax = 1024;  // persistent workgroups of a chain launch (about; at least one per entry)
int part_chain_counters(int nent, int np);
bool part_fits(const Geom& g, const SolveLayout& L);
template <typename R>
hipError_t launch_part_phi(const Geom& g, const SolveLayout& L, const PartLayout& pl,
                           const typename Cplx<R>::T* mf, const int16_t* pf, const int32_t* pflag,
                           const typename Cplx<R>::T* mb, typename Cplx<R>::T* phi_f, typename Cplx<R>::T* phi_b,
                           int nsub, hipStream_t st);
template <typename R>
hipError_t launch_fwd_part(const Geom& g, const SolveLayout& L, const PartLayout& pl, const Entry* ent, int nent,
                           const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mf, const int16_t* pf,
                           const int32_t* pflag, const typename Cplx<R>::T* phi_f, const SolveIO& io,
                           typename Cplx<R>::T* rb, typename Cplx<R>::T* y2, typename Cplx<R>::T* sig,
                           typename Cplx<R>::T* tt, PartWait& pw, hipStream_t st);
template <typename R>
hipError_t launch_bwd_part(const Geom& g, const SolveLayout& L, const PartLayout& pl, const Entry* ent, int nent,
                           const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mb,
                           const typename Cplx<R>::T* phi_b, const SolveIO& io, const typename Cplx<R>::T* y2,
                           typename Cplx<R>::T* rb, typename Cplx<R>::T* sig, typename Cplx<R>::T* tt, PartWait& pw,
                           hipStream_t st);

// The same solves for tiles of up to 16 entries of one subdomain (tiles[t] = {first entry, count},
// entries of a tile consecutive and with the same subdomain), 16 right-hand sides per workgroup on
// MFMA; results and outputs as launch_fwd / launch_bwd.  piv: some subdomain has row interchanges.
// sink: nblk * nb elements that absorb the stores of lanes without a right-hand side.
bool trisolve_mm_fits(const SolveLayout& L, size_t elem);
template <typename R>
hipError_t launch_fwd_mm(const Geom& g, const SolveLayout& L, const Entry* ent, const int2* tiles, int ntiles,
                         const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mf, const int16_t* pf,
                         const int32_t* pflag, bool piv, const SolveIO& io, typename Cplx<R>::T* ybuf,
                         typename Cplx<R>::T* sink, hipStream_t st);
template <typename R>
hipError_t launch_bwd_mm(const Geom& g, const SolveLayout& L, const Entry* ent, const int2* tiles, int ntiles,
                         const FaceTab* ft, const IfCoef* coef, const typename Cplx<R>::T* mb, const SolveIO& io,
                         typename Cplx<R>::T* ybuf, typename Cplx<R>::T* sink, hipStream_t st);

// Krylov helpers on [ncol][n] column blocks (complex128)
hipError_t launch_multidot(const double2* V, size_t vstride, int nvec, const double2* w, int n, int ncol,
                           double2* partial, int nchunk, hipStream_t st);
hipError_t launch_reduce_partials(const double2* partial, int nvec, int ncol, int nchunk, double2* out,
                                  size_t out_stride, double2 scale, hipStream_t st);
hipError_t launch_update(double2* w, const double2* V, size_t vstride, int nvec, const double2* h,
                         size_t h_stride, double2 alpha, int n, int ncol, hipStream_t st);
// fused forms: h = sum of the partials (chunk order) inside the update, |w|^2 partials per
// update workgroup, then the norm and the scaling in one launch
bool krylov_fusable(int nvec, int nchunk, int n);
hipError_t launch_update_reduce(double2* w, const double2* V, size_t vstride, int nvec, const double2* partial,
                                int nchunk, double2* h_out, size_t h_stride, double2 alpha, int n, int ncol,
                                double* npart, hipStream_t st);
hipError_t launch_scale_reduce(double2* dst, const double2* src, const double* npart, double* nrm_out, int n, int ncol,
                               hipStream_t st);
// s-step Arnoldi: block Gram-Schmidt of up to kSstepMax new vectors against at most
// kSstepMaxBasis - kSstepMax earlier ones (inner products, Cholesky of the projected Gram matrix,
// update in place); per column a coefficient record of kSstepCoefLd entries (R, R^{-1}, the first
// failed pivot, C)
constexpr int kSstepMax = 8;
constexpr int kSstepMaxBasis = 64;
constexpr int kSstepCoefLd = 129 + kSstepMaxBasis * kSstepMax;
int bgs_positions_per_wg(int n, int ncol, int wgs);
int bgs_chunks(int n, int ncol, int wgs);
size_t bgs_partial_elems(int n, int ncol);
hipError_t launch_bgs(double2* V, size_t vstride, int k1, int sb, int n, int ncol, double2* part, size_t part_elems,
                      double2* coef, int ldc, hipStream_t st);
// Gram-Schmidt with delayed reorthogonalisation: one pass of inner products, one update pass
bool dcgs_fits(int m, int nchunk);
hipError_t launch_dots2(const double2* V, size_t vstride, int nv, const double2* x, const double2* w, int n, int ncol,
                        double2* partial, int nchunk, hipStream_t st);
hipError_t launch_dcgs_update(const double2* V, size_t vstride, int nv, double2* x, double2* xn, const double2* w,
                              const double2* partial, int nchunk, double2* hout, int ld, int n, int ncol,
                              bool publish_only, hipStream_t st);
hipError_t launch_norms(const double2* w, int n, int ncol, double* partial, int nchunk, hipStream_t st);
hipError_t launch_reduce_norms(const double* partial, int ncol, int nchunk, double* out, hipStream_t st);
hipError_t launch_scale_by_inv(double2* dst, const double2* src, const double* nrm, int n, int ncol,
                               hipStream_t st);
hipError_t launch_axpby(double2* y, const double2* x, double2 a, double2 b, size_t n, hipStream_t st);
hipError_t launch_copy(double2* dst, const double2* src, size_t n, hipStream_t st);
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t st);
hipError_t launch_add_ranges(double2* y, const double2* x, const int32_t* ranges, int nranges, int nif, int ncol,
                             hipStream_t st);

hipError_t launch_source_flags(const Geom& g, const double2* f, int nrhs, int32_t* nz, hipStream_t st);
// dense scattering operators (row-block layout t_index); every entry of one launch carries the
// same face mask; rblist: distinct row blocks holding rows of the masked faces
// outgoing traces of masked faces from whole local fields x64 [entry][nloc] (the band rows of the
// transmission condition), plus the field outputs of io
hipError_t launch_emit_traces(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfBand* band,
                              const SolveIO& io, const double2* x64, hipStream_t st);
hipError_t launch_build_T(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfBand* band,
                          const double2* ybuf, size_t ystride, double2* T, hipStream_t st);
template <typename C>
hipError_t launch_scatter_apply(const Geom& g, const Entry* ent, int nent, int mask, const int32_t* rblist, int nrb,
                                const FaceTab* eft, const C* T, const SolveIO& io, hipStream_t st,
                                hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr, const StepArgs* sa = nullptr);
// dataflow sweep launch: ctr = [ticket, counters...] (zero at entry), ctr_next is zeroed for the
// next launch; err receives 1 if a dependency wait exceeded spin_limit polls; the waits of
// task stall_task (-1: none) need one completion more than exists (error-path tests)
template <typename C>
hipError_t launch_sweep_df(const Geom& g, const DfTask* tasks, int ntasks, const FaceTab* ft, const C* T,
                           const DfArgs& A, int32_t* ctr, int32_t* ctr_next, int nctr, int32_t* err, int spin_limit,
                           int stall_task, int grid, hipStream_t st);
int sweep_df_occupancy(int L, bool c64);

// dense lifting operators W[s][p][row] = -sigma_row x_row[p] / inj_row from the unit-datum
// solves of a batch of entries (s, col = row); b = W_s^T f_s for the (s, rhs) with a source
hipError_t launch_build_W(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfCoef* coef,
                          const double2* ybuf, size_t ystride, double2* W, hipStream_t st);
int lift_chunks(const Geom& g, int pchunk);
// the first pass of launch_lift_dense alone: part[(r, s, chunk)][row] = sum over the chunk's nodes of W f
hipError_t launch_lift_partials(const Geom& g, const double2* W, const double2* f, const int32_t* nz, int nrhs,
                                int pchunk, double2* part, hipStream_t st);
hipError_t launch_lift_dense(const Geom& g, const FaceTab* ft, const IfBand* band, const double2* W, const double2* f,
                             const int32_t* nz, int nrhs, int pchunk, double2* part, double2* b, hipStream_t st);
// many right-hand sides: the same transmission part as one complex matrix product per
// subdomain on MFMA (Gbuf: ndom * L * round16(nrhs) entries of workspace)
hipError_t launch_recon_mm(const Geom& g, const IfCoef* coef, const FaceTab* ft, const double2* W, const double2* gin,
                           const int32_t* nz, int nrhs, double2* Gbuf, double2* u, hipStream_t st);
// u += A_s^{-1} B_s g through W (u is read only where nz marks a source: it then holds
// A_s^{-1} f_s; elsewhere it is overwritten)
hipError_t launch_recon_dense(const Geom& g, const FaceTab* ft, const IfCoef* coef, const double2* W,
                              const double2* gin, const int32_t* nz, int nrhs, double2* u, hipStream_t st);

// many right-hand sides: gather the incoming data G[j][col][r] of subdomains subs[j] (in the element
// type GT); OUT = T_s[masked rows, :] G_s on MFMA (complex128 operators on f64 MFMA, complex64 on
// f32), with G_s from the gathered tiles G (variants 0-2: k-steps per batch 2, 4, 8) or straight
// from the interface vector gin [nrhs][nif] (variants 3-5); variants 6-11 as 0-5 with the
// right-hand sides split over two groups of wavefronts
template <typename GT>
hipError_t launch_gather_incoming(const Geom& g, const int32_t* subs, int nsub, const FaceTab* ft, const double2* gin,
                                  int nrhs, int rpad, GT* G, hipStream_t st);
// tiles[dst[q] + r] = gin[r][pos[q]] for r < nrhs (zeros up to rpad): the gathered tiles of a pass
template <typename GT>
hipError_t launch_pregather(const int64_t* dst, const int32_t* pos, int njobs, const double2* gin, int nif, int nrhs,
                            int rpad, GT* tiles, hipStream_t st);
template <typename C>
hipError_t launch_scatter_mm(const Geom& g, const int32_t* subs, int nsub, int mask, const FaceTab* ft, const C* T,
                             const double2* gin, const C* G, int nrhs, int rpad, const SolveIO& io, hipStream_t st,
                             int variant);
// Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b % 8), each XCD with its own L2.
// Tile index of workgroup b such that XCD x works on one contiguous run of tiles (a bijection of
// [0, n)): consecutive tiles that read the same data (the factors of one subdomain, its incoming
// data) then share an L2, and the data are fetched once per XCD.
__device__ inline int xcd_tile(int b, int n) {
  const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + k;
}

// variants 0-11: k-steps per batch 2, 4, 8; gathered or direct; one or two wave groups;
// 12-15: a register ring of 4 or 8 k-steps over all faces, gathered or direct, two wave groups;
// 16, 17: gathered with 4 k-steps per batch, direct with 2, two wave groups; 12-17 with the tiles
// of one subdomain on one XCD; 18-21: eight wavefronts splitting the k range, one group, 2 or 4
// k-steps per batch, gathered (18, 19) or direct (20, 21)
constexpr int kMmVariants = 22;
__host__ __device__ inline bool mm_variant_gathered(int v) {
  return v < 12 ? (v % 6 < 3) : v < 16 ? (v < 14) : v < 18 ? (v == 16) : (v < 20);
}

// gradient / misc
hipError_t launch_gather_receivers(const double2* u, const int32_t* rec, int nrec, int npts, const double2* d,
                                   double2* resid, int nsrc, hipStream_t st);
hipError_t launch_spread_adjoint(const double2* resid, const int32_t* rec, int nrec, int npts, double2* f_adj,
                                 int nsrc, hipStream_t st);
hipError_t launch_grad_accumulate(const Geom& g, const double* m, const double2* u, const double2* mu, int nsrc,
                                  double* grad, hipStream_t st);
// global residual sums of r = f - A u (|r|^2 and |f|^2 per right-hand side into sums[2 nrhs]);
// part holds volume_residual_blocks(g) * 2 doubles per right-hand side
int volume_residual_blocks(const Geom& g);
hipError_t launch_volume_residual(const Geom& g, const double* m, const double2* f, const double2* u, int nrhs,
                                  double* part, double* sums, hipStream_t st);
// the allocation-free variant: partial pairs in the library's static per-device scratch (its
// address resolved once per device, with that device current, by volume_residual_scratch_init),
// relres[nrhs] left on the device; hipErrorInvalidValue for nrhs outside 1..HBJ_VR_NOALLOC_MAX_RHS,
// hipErrorNotInitialized when the scratch address of dev was never resolved
hipError_t volume_residual_scratch_init(int dev);
hipError_t launch_volume_residual_noalloc(int dev, const Geom& g, const double* m, const double2* f,
                                          const double2* u, int nrhs, double* relres, hipStream_t st);
// Pade transmission, dense form: face blocks (rho, Sigma, J, C per interface face, pade_fb_per_sub
// entries per subdomain) on the host; on the device G^-1 and the operators T, the lifting and the
// reconstruction data (see k_pade.hip)
size_t pade_fb_per_sub(const Geom& g);
int pade_face_blocks(const Geom& g, const FaceTab* ft_host, const double* m_host, const IfCoef* coef_host,
                     int npade, double phi, double2* rho, double2* sigma, double2* inj, double2* corr);
hipError_t launch_pade_T(const Geom& g, const FaceTab* ft, const double2* W, const double2* fbP, const double2* fbS,
                         const double2* fbJ, const double2* fbC, double2* Ginv, double2* work, int32_t* piv,
                         int32_t* info, double2* T, hipStream_t st);
hipError_t launch_pade_lift(const Geom& g, const FaceTab* ft, const double2* fbS, const double2* Ginv,
                            const int32_t* nz, const double2* part, int nchunk, int nrhs, double2* b, hipStream_t st);
hipError_t launch_pade_recon_prep(const Geom& g, const FaceTab* ft, const IfCoef* coef, const double2* fbJ,
                                  const double2* fbC, const double2* Ginv, const double2* gin, const int32_t* nz,
                                  const double2* u, int nrhs, double2* qbuf, double2* gt, hipStream_t st);
// ratio[e] = ||r_e|| / ||b_e|| over the nloc entries of each of nent local vectors
hipError_t launch_entry_ratio(const double2* r, const double2* b, int nloc, int nent, double* ratio, hipStream_t st);
hipError_t launch_local_residual(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfBand* band,
                                 const double2* diag, const double2* rhs64, const double2* x64, double2* r64,
                                 hipStream_t st);
