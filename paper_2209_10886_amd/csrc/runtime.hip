// Host runtime of libhbj: decomposition tables, sweep scheduler, (F)GMRES driver, C ABI.
//
// Layout (paper Sec. 2).  Subdomains are multi-indices i = (i1, i2), 1-based, ordered
// by the lexicographic order of Definition 1 (|i|_1 first, then i1).  Ordered pairs
// (i, j), j a neighbour of i, are ordered by Definition 2; the map m numbers them and
// block m(i, j) of the interface vector holds the data i receives from j.  Groups V_a
// (receiver on anti-diagonal a, Sec. 5) are contiguous ranges of that order.
//
// Sweeps (Secs. 5-6).  A pass is a list of lockstep steps; each step is one batched
// launch of local solves over the subdomains of the active anti-diagonals, whose
// outgoing traces are added into the blocks of the next anti-diagonal.  SGS is the
// single interval [2, N_g + 1]; block Jacobi cuts it into closed intervals of
// bj_width anti-diagonals that advance together (2 bj_width steps per application).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "hbj_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(HBJ_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

typedef std::complex<double> zc;

// faces written by a forward sweep step (toward +x, +y) and by a backward step (toward -x, -y)
constexpr int kMaskFwd = (1 << FACE_E) | (1 << FACE_N);
constexpr int kMaskBwd = (1 << FACE_W) | (1 << FACE_S);

// launch shapes of a batch of banded local solves: one workgroup per solve at the prefetch depth
// variants of the solve kernels, then 16 right-hand sides of one subdomain per workgroup on MFMA,
// then each solve split over several workgroups (runs of column blocks)
constexpr int kShapeMfma = kSolveDepthVariants;
constexpr int kShapePart = kSolveDepthVariants + 1;
constexpr int kSolveShapes = kSolveDepthVariants + 2;
constexpr int kPartDefault = 16;  // runs per split solve (hbj_set_solve_partitions)

constexpr int kMatrixRhs = 4;  // from this many right-hand sides on, the operators run as MFMA products

struct Step {
  size_t first;  // offset into the schedule's device entry array
  int count;
  double dense_elems = 0;  // dense operator entries read by the step (rows x columns)
  size_t sub_first = 0;    // offset into the schedule's subdomain list (one per subdomain)
  int sub_count = 0;
  size_t tile_first = 0;   // offset into the schedule's tile list (banded solves on MFMA)
  int tile_count = 0;
  int sarg = -1;           // the step's tables by value (dense operators), index into Schedule::sargs
};

// All launches for a given number of right-hand sides.
struct Schedule {
  int nrhs = 0;
  Entry* dev = nullptr;
  FaceTab* eft = nullptr;  // the face table of each entry's subdomain, one per entry (same indexing)
  size_t all_first = 0;  // every subdomain, all faces
  int all_count = 0;
  double all_dense_elems = 0;
  int32_t* subs = nullptr;  // device subdomain lists of the steps (many right-hand sides)
  size_t all_sub_first = 0;
  int all_sub_count = 0;
  int2* tiles = nullptr;  // {first entry relative to the step's first, count}: runs of one subdomain, <= 16
  size_t all_tile_first = 0;
  int all_tile_count = 0;
  std::vector<Step> fwd, bwd;  // preconditioner passes
  std::vector<StepArgs> sargs;
  // the operator (I - S) z applied while the backward pass still runs (dense operators, few
  // right-hand sides, default readings): after backward step k, the operator rows of the
  // subdomains whose incoming and outgoing data the pass has finalised by then, entries
  // [ov_first[k], ov_first[k] + ov_count[k]) of dev/eft (mask 0xF)
  bool ov_ok = false;
  std::vector<size_t> ov_first;
  std::vector<int> ov_count;
  // no step of either pass holds two neighbouring subdomains (a pass can then run in place)
  bool steps_apart = false;
  std::vector<int32_t> subs_host;  // host copy of subs
  // chained sweep steps (matrix-product path, passes in place): per pass, the gathered tile of
  // every step in one buffer (tile_off), filled at the pass start for the positions the previous
  // step does not write (jobs: destination entry, position) and by the previous step's outputs
  // for the others (cmap: per step, position -> slot in the next step's tile, -1 if none)
  struct Chain {
    bool built = false, ok = false;
    std::vector<size_t> tile_off;  // elements of the tile buffer, one entry per step and the end
    int32_t* cmap = nullptr;       // [steps][nif]
    int64_t* jdst = nullptr;
    int32_t* jpos = nullptr;
    int njobs = 0;
  };
  Chain chain[2];  // forward, backward
  // dataflow launches (dense form): task lists per kind, double-buffered completion counters
  struct DfPlan {
    bool built = false;
    DfTask* dev = nullptr;
    int ntasks = 0;
    double tbytes = 0;  // operator bytes streamed by the launch
    double flops = 0;
  };
  DfPlan df[5];
  int32_t* df_ctr = nullptr;  // two regions of df_nctr ints: [ticket, counters...]
  int df_nctr = 0;
  int df_parity = 0;
};
constexpr int kLiftChunk = 128;                         // nodes per lifting workgroup
constexpr size_t kLiftPartialElems = (size_t)16 << 20;  // lifting partials per batch (256 MB)
// dataflow plan kinds
enum { DF_FWD = 0, DF_BWD = 1, DF_PC = 2, DF_PC_OP = 3, DF_OP = 4 };
constexpr int kDfSpinDefault = 1 << 19;  // polls of about 1 us: well under a second

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return hipSuccess;
  return hipMalloc((void**)p, n * sizeof(T));
}

struct Gmres;
void destroy_gmres(Gmres* g);

}  // namespace

struct hbj_ctx {
  hbj_problem P{};
  hipStream_t st = nullptr;
  Geom g{};
  SolveLayout L{};
  int ndom = 0, ne = 0, ng = 0;
  int bj_width = 0;
  std::vector<std::pair<int, int>> fblocks, bblocks;  // intervals of anti-diagonals
  std::vector<FaceTab> ft_host;
  std::vector<int> grp_lo, grp_hi;  // interface positions of group a (index a)
  // device tables
  FaceTab* ft = nullptr;
  IfCoef* coef = nullptr;
  IfBand* band = nullptr;  // R / Sigma rows and tangential weights of the transmission condition
  int32_t* pos_tab = nullptr;
  double* m = nullptr;
  double2* diag = nullptr;
  int32_t* ranges_f = nullptr;  // additive reading: shared groups of the forward intervals
  int32_t* ranges_b = nullptr;
  int nranges_f = 0, nranges_b = 0;
  // factors
  double2* ab = nullptr;
  int32_t* ipiv = nullptr;
  int32_t* info = nullptr;
  double2* mf64 = nullptr;
  double2* mb64 = nullptr;
  int16_t* pf = nullptr;
  int32_t* pflag = nullptr;
  float2* mf32 = nullptr;
  float2* mb32 = nullptr;
  double2* Wl = nullptr;    // dense lifting operators [ndom][n_loc][L] (null: banded lifting)
  hipStream_t side = nullptr;  // source part of the reconstruction, overlapped with GMRES
  hipStream_t opst = nullptr;  // operator rows overlapped with the backward pass
  std::vector<hipEvent_t> ov_ev;  // one per backward step, and the join
  bool op_overlap = false;        // measured slower: each stream-to-stream wait costs ~19 us here
  bool chain_ok = true;           // chained sweep steps where they apply (hbj_set_step_chaining)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  void* ybuf_side = nullptr;
  size_t ybuf_side_bytes = 0;
  double2* lpart = nullptr; // lifting partial sums
  size_t lpart_cap = 0;
  double2* T64 = nullptr;  // dense scattering operators [ndom][t_rows][L] (row blocks, t_index)
  float2* T32 = nullptr;
  int32_t* rbl = nullptr;  // stepped launches: row blocks of the forward, backward and full masks
  int rbl_off[3] = {0, 0, 0}, rbl_n[3] = {0, 0, 0};
  std::vector<int32_t> rbl_host;
  int32_t* df_err = nullptr;  // dataflow dependency-wait error flag
  int df_grid = 0;            // persistent workgroups per dataflow launch
  int df_spin = kDfSpinDefault;
  int df_stall = -1;
  bool dense = false;
  bool factored = false;
  int zero_sub = -1, zero_row = -1;
  // schedules
  std::map<int, std::unique_ptr<Schedule>> sched;
  // workspace
  void* ybuf = nullptr;
  size_t ybuf_bytes = 0;
  double2* rhs64 = nullptr;  // mixed: local right-hand sides / residuals
  double2* x64 = nullptr;
  double2* xtr = nullptr;  // local fields of a banded batch whose traces follow the second-order condition
  size_t xtr_entries = 0;
  double2* r64 = nullptr;
  size_t loc64_entries = 0;
  double2* Gbuf = nullptr;  // gathered incoming data for the many-right-hand-side operators
  size_t Gbuf_cap = 0;
  void* chain_buf = nullptr;  // gathered tiles of a chained preconditioner pass
  size_t chain_cap = 0;       // bytes
  // autotuned tile depth of the many-right-hand-side operator kernel, per (precision, stage kind):
  // [complex128 steps, complex128 operator, complex64 steps, complex64 operator]; -1 = not tuned
  int mm_variant[4] = {-1, -1, -1, -1};
  float mm_us[4][kMmVariants] = {};
  // autotuned launch shapes of the banded solve batches, per batch class (its cache key)
  struct SolveChoice {
    int shape = 0;
    float us[kSolveShapes] = {};
  };
  std::map<std::string, SolveChoice> solve_choice;
  int solve_shape_fixed = -1;  // hbj_set_solve_tuning: -1 = by timing
  // split solves: runs per solve, the runs' transfer matrices per precision [complex128, complex64]
  // (formed for the factorisation of graph_epoch), the forward results and the run states
  int part_np = kPartDefault;
  void* phi[2] = {nullptr, nullptr};
  size_t phi_bytes[2] = {0, 0};
  int phi_epoch[2] = {-1, -1};
  int phi_np[2] = {0, 0};
  void* part_y2 = nullptr;
  size_t part_y2_bytes = 0;
  void* part_st = nullptr;
  size_t part_st_bytes = 0;
  int32_t* part_ctr = nullptr;  // chain completion counters (two regions) and their wait error flag
  int part_nctr = 0;
  int part_parity = 0;
  int32_t* part_err = nullptr;
  std::string arch;            // device architecture name (cache keys)
  int32_t* nzf = nullptr;   // per (rhs, subdomain) nonzero-source flags for the lifting
  size_t nzf_cap = 0;
  double2* pc_y = nullptr;  // preconditioner pass buffers [nrhs][nif]
  double2* pc_t = nullptr;
  size_t pc_cols = 0;
  // GMRES workspace kept across solves, and the HIP graphs of its iterations
  Gmres* gm = nullptr;
  bool use_graphs = false;  // eager launches measured faster once step j+1 is queued ahead
  int orth = HBJ_ORTH_AUTO;      // Gram-Schmidt variant of the Arnoldi steps
  int sstep_block = kSstepMax;   // steps per block of the s-step Arnoldi cycle
  bool interchanges = true;      // some subdomain factorisation has row interchanges (set by hbj_factor)
  int msolve = HBJ_MSOLVE_MFMA;  // banded solves of many right-hand sides per subdomain on MFMA
  int graph_epoch = 0;           // bumped when captured operands change (a new factorisation)
  hipStream_t cap = nullptr;     // capture stream (graphs are replayed on st)
  // profiling
  bool prof = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hbj_kernel_stat ks[HBJ_K_NCLASS]{};
  int64_t local_solves = 0;
  int last_ir = 0;             // solves of the last refined local solve batch (mixed banded operator)
  double last_ir_resid = 0.0;  // its largest final relative local residual
  int ir_max = 0;              // the same, maximised over the current solve
  double ir_resid_max = 0.0;
  double* ir_ratio = nullptr;  // per-entry relative residuals of the refinement
  size_t ir_ratio_cap = 0;
  // volume residual: per-workgroup partial sums and the per-right-hand-side totals
  double* vr_part = nullptr;
  size_t vr_cap = 0;  // right-hand sides the buffer holds
  int dev = 0;        // device current at hbj_setup (the allocation-free residual's scratch)
  // Pade transmission (dense form): face blocks rho, Sigma, J and the correction C of every
  // subdomain, G^-1 = (I + C M)^-1 per subdomain, and the reconstruction data workspace
  double2* pade_P = nullptr;
  double2* pade_S = nullptr;
  double2* pade_J = nullptr;
  double2* pade_C = nullptr;
  double2* Ginv = nullptr;
  double2* pade_gt = nullptr;
  size_t pade_gt_cap = 0;

  ~hbj_ctx();
};

namespace {

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

}  // namespace

hbj_ctx::~hbj_ctx() {
  destroy_gmres(gm);
  gm = nullptr;
  if (cap) (void)hipStreamDestroy(cap);
  for (auto& kv : sched) {
    dfree(kv.second->dev);
    dfree(kv.second->eft);
    dfree(kv.second->subs);
    dfree(kv.second->tiles);
    for (auto& pl : kv.second->df) dfree(pl.dev);
    dfree(kv.second->df_ctr);
    for (auto& ch : kv.second->chain) {
      dfree(ch.cmap);
      dfree(ch.jdst);
      dfree(ch.jpos);
    }
  }
  dfree(chain_buf);
  dfree(rbl);
  dfree(df_err);
  dfree(vr_part);
  dfree(ir_ratio);
  for (void* p : {(void*)pade_P, (void*)pade_S, (void*)pade_J, (void*)pade_C, (void*)Ginv, (void*)pade_gt}) dfree(p);
  for (void* p : {(void*)ft, (void*)coef, (void*)band, (void*)pos_tab, (void*)m, (void*)diag, (void*)ranges_f, (void*)ranges_b,
                  (void*)ab, (void*)ipiv, (void*)info, (void*)mf64, (void*)mb64, (void*)pf, (void*)pflag, (void*)mf32, (void*)mb32, (void*)T64, (void*)T32, (void*)Wl, (void*)lpart,
                  ybuf, (void*)nzf, (void*)Gbuf, (void*)rhs64, (void*)x64, (void*)xtr, (void*)r64, (void*)pc_y, (void*)pc_t})
    dfree(p);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (side) {
    (void)hipStreamSynchronize(side);
    (void)hipStreamDestroy(side);
  }
  if (opst) {
    (void)hipStreamSynchronize(opst);
    (void)hipStreamDestroy(opst);
  }
  for (hipEvent_t e : ov_ev) (void)hipEventDestroy(e);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  dfree(ybuf_side);
  dfree(phi[0]);
  dfree(phi[1]);
  dfree(part_y2);
  dfree(part_st);
  dfree(part_ctr);
  dfree(part_err);
}

namespace {

// ---------------------------------------------------------------------------
// paper Sec. 2: orders and the pair map m
// ---------------------------------------------------------------------------
struct MI {
  int i1, i2;
};
inline bool mi_less(MI a, MI b) {  // Definition 1
  const int na = a.i1 + a.i2, nb = b.i1 + b.i2;
  return na < nb || (na == nb && a.i1 < b.i1);
}
inline bool mi_eq(MI a, MI b) { return a.i1 == b.i1 && a.i2 == b.i2; }
inline int sub_index(const hbj_ctx* c, MI a) { return (a.i2 - 1) * c->P.n1 + (a.i1 - 1); }

// Builds face tables, pos_tab and group ranges on the host.
void build_layout(hbj_ctx* c, std::vector<int32_t>& pos_tab) {
  const int n1 = c->P.n1, n2 = c->P.n2;
  struct Pair {
    MI i, j;
    int face;  // face of i through which j is seen
  };
  std::vector<Pair> pairs;
  for (int i1 = 1; i1 <= n1; ++i1)
    for (int i2 = 1; i2 <= n2; ++i2) {
      const MI i{i1, i2};
      const MI nb[4] = {{i1 - 1, i2}, {i1 + 1, i2}, {i1, i2 - 1}, {i1, i2 + 1}};
      for (int f = 0; f < 4; ++f)
        if (nb[f].i1 >= 1 && nb[f].i1 <= n1 && nb[f].i2 >= 1 && nb[f].i2 <= n2) pairs.push_back({i, nb[f], f});
    }
  std::sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {  // Definition 2
    if (!mi_eq(a.i, b.i)) return mi_less(a.i, b.i);
    return mi_less(a.j, b.j);
  });
  c->ft_host.assign(c->ndom, FaceTab{{-1, -1, -1, -1}, {-1, -1, -1, -1}});
  std::map<std::pair<int, int>, int> off;  // (receiver, sender) -> offset
  int pos = 0;
  c->grp_lo.assign(c->ng + 3, -1);
  c->grp_hi.assign(c->ng + 3, -1);
  pos_tab.clear();
  for (const Pair& p : pairs) {
    const int len = (p.face < 2) ? c->g.sny : c->g.snx;
    const int si = sub_index(c, p.i), sj = sub_index(c, p.j);
    off[{si, sj}] = pos;
    c->ft_host[si].in_off[p.face] = pos;
    const int a = p.i.i1 + p.i.i2;
    if (c->grp_lo[a] < 0) c->grp_lo[a] = pos;
    c->grp_hi[a] = pos + len;
    for (int e = 0; e < len; ++e) {
      pos_tab.push_back(si);
      pos_tab.push_back(p.face);
      pos_tab.push_back(e);
      pos_tab.push_back(0);
    }
    pos += len;
  }
  c->g.nif = pos;
  // out offsets: face f of i sends into block m(j, i)
  for (int s = 0; s < c->ndom; ++s) {
    const int i1 = s % n1 + 1, i2 = s / n1 + 1;
    const MI nb[4] = {{i1 - 1, i2}, {i1 + 1, i2}, {i1, i2 - 1}, {i1, i2 + 1}};
    for (int f = 0; f < 4; ++f) {
      if (c->ft_host[s].in_off[f] < 0) continue;
      c->ft_host[s].out_off[f] = off[{sub_index(c, nb[f]), s}];
    }
  }
}

std::vector<int> antidiag_subdomains(const hbj_ctx* c, int a) {
  std::vector<int> out;
  for (int i1 = 1; i1 <= c->P.n1; ++i1) {
    const int i2 = a - i1;
    if (i2 >= 1 && i2 <= c->P.n2) out.push_back(sub_index(c, MI{i1, i2}));
  }
  return out;
}

// closed intervals of Sec. 6
void build_blocks(hbj_ctx* c) {
  const int w = c->bj_width;
  const int p = (c->ng - 1 + w - 1) / w;
  c->fblocks.clear();
  c->bblocks.clear();
  for (int b = 1; b <= p; ++b) {
    c->fblocks.push_back({2 + (b - 1) * w, std::min(2 + b * w, c->ng + 1)});
    c->bblocks.push_back({std::max(2, (1 + c->ng) - b * w), (1 + c->ng) - (b - 1) * w});
  }
}

// runs of at most 16 consecutive entries with one subdomain, as {first - base, count}
void append_tiles(const std::vector<Entry>& ent, size_t first, int count, std::vector<int2>& tiles) {
  for (int q = 0; q < count;) {
    int n = 1;
    while (q + n < count && n < 16 && ent[first + q + n].s == ent[first + q].s) ++n;
    tiles.push_back(make_int2(q, n));
    q += n;
  }
}

// Which operator rows may run while the backward pass is still under way.  A backward step writes,
// per entry (subdomain s, faces W and S), the outgoing data of s toward its W and S neighbours and
// (copy mode: the pass output is not pre-filled) s's own incoming positions on those faces; every
// position of the pass output is written by exactly one step.  The operator rows of s read the
// pass output at s's incoming positions and at its outgoing positions (the base of z - S z there),
// so they can run once the last step writing any of those positions has run.  Entries of mask 0xF,
// grouped by that step, are appended to ent; a position that no step writes disables the overlap.
void plan_operator_overlap(const hbj_ctx* c, Schedule& S, std::vector<Entry>& ent) {
  const Geom& g = c->g;
  std::vector<int> wstep(g.nif, -1);
  for (size_t k = 0; k < S.bwd.size(); ++k) {
    const Step& st = S.bwd[k];
    for (int q = 0; q < st.count; ++q) {
      const Entry& e = ent[st.first + q];
      if (e.rhs != 0) continue;  // the same positions for every right-hand side
      const FaceTab& F = c->ft_host[e.s];
      for (int f = 0; f < 4; ++f) {
        if (!((e.mask >> f) & 1)) continue;
        const int len = face_len(g, f);
        for (int off : {F.out_off[f], F.in_off[f]})
          if (off >= 0)
            for (int i = 0; i < len; ++i) wstep[off + i] = std::max(wstep[off + i], (int)k);
      }
    }
  }
  const int nk = (int)S.bwd.size();
  std::vector<std::vector<int>> by_step(nk);
  for (int s = 0; s < c->ndom; ++s) {
    const FaceTab& F = c->ft_host[s];
    int ready = -1;
    for (int f = 0; f < 4; ++f) {
      const int len = face_len(g, f);
      for (int off : {F.out_off[f], F.in_off[f]}) {
        if (off < 0) continue;
        for (int i = 0; i < len; ++i) {
          if (wstep[off + i] < 0) return;  // not written by the pass: keep the operator after it
          ready = std::max(ready, wstep[off + i]);
        }
      }
    }
    by_step[std::max(ready, 0)].push_back(s);
  }
  for (int k = 0; k < nk; ++k) {
    S.ov_first.push_back(ent.size());
    for (int s : by_step[k])
      for (int r = 0; r < S.nrhs; ++r) ent.push_back(Entry{s, r, 0, 0xF});
    S.ov_count.push_back((int)(ent.size() - S.ov_first.back()));
  }
  S.ov_ok = true;
}

int build_schedule(hbj_ctx* c, int nrhs, Schedule** out) {
  auto it = c->sched.find(nrhs);
  if (it != c->sched.end()) {
    *out = it->second.get();
    return HBJ_OK;
  }
  auto S = std::make_unique<Schedule>();
  S->nrhs = nrhs;
  std::vector<Entry> ent;
  S->all_first = 0;
  auto dense_elems = [&](const Entry& e) {
    const FaceTab& F = c->ft_host[e.s];
    double rows = 0, cols = 0;
    for (int f = 0; f < 4; ++f) {
      if (F.in_off[f] < 0) continue;
      cols += face_len(c->g, f);
      if ((e.mask >> f) & 1) rows += face_len(c->g, f);
    }
    return rows * cols;
  };
  std::vector<int32_t> subs;
  for (int s = 0; s < c->ndom; ++s)
    for (int r = 0; r < nrhs; ++r) ent.push_back(Entry{s, r, 0, 0xF});
  S->all_count = (int)ent.size();
  S->all_sub_first = 0;
  for (int s = 0; s < c->ndom; ++s) subs.push_back(s);
  S->all_sub_count = c->ndom;
  for (const Entry& e : ent) S->all_dense_elems += dense_elems(e);
  const int maskF = kMaskFwd, maskB = kMaskBwd;
  if (c->P.precond != HBJ_PC_NONE && c->ndom > 1) {
    int nsteps = 0;
    for (auto& b : c->fblocks) nsteps = std::max(nsteps, b.second - b.first);
    for (int t = 1; t <= nsteps; ++t) {
      Step st{ent.size(), 0};
      st.sub_first = subs.size();
      for (auto& b : c->fblocks) {
        if (b.first + t > b.second) continue;
        for (int s : antidiag_subdomains(c, b.first + t - 1)) {
          subs.push_back(s);
          for (int r = 0; r < nrhs; ++r) ent.push_back(Entry{s, r, t == 1 ? 0 : 1, maskF});
        }
      }
      st.sub_count = (int)(subs.size() - st.sub_first);
      st.count = (int)(ent.size() - st.first);
      for (size_t q = st.first; q < ent.size(); ++q) st.dense_elems += dense_elems(ent[q]);
      S->fwd.push_back(st);
    }
    nsteps = 0;
    for (auto& b : c->bblocks) nsteps = std::max(nsteps, b.second - b.first);
    for (int t = 1; t <= nsteps; ++t) {
      Step st{ent.size(), 0};
      st.sub_first = subs.size();
      for (auto& b : c->bblocks) {
        if (b.second - t < b.first) continue;
        for (int s : antidiag_subdomains(c, b.second - t + 1)) {
          subs.push_back(s);
          for (int r = 0; r < nrhs; ++r) ent.push_back(Entry{s, r, t == 1 ? 0 : 1, maskB});
        }
      }
      st.sub_count = (int)(subs.size() - st.sub_first);
      st.count = (int)(ent.size() - st.first);
      for (size_t q = st.first; q < ent.size(); ++q) st.dense_elems += dense_elems(ent[q]);
      S->bwd.push_back(st);
    }
  }
  {
    std::vector<int> stamp(c->ndom, -1);
    bool apart = true;
    int id = 0;
    for (auto* v : {&S->fwd, &S->bwd})
      for (const Step& st : *v) {
        for (int q = 0; q < st.sub_count; ++q) stamp[subs[st.sub_first + q]] = id;
        for (int q = 0; q < st.sub_count && apart; ++q) {
          const int sd = subs[st.sub_first + q];
          const int i1 = sd % c->P.n1 + 1, i2 = sd / c->P.n1 + 1;
          const MI nb[4] = {{i1 - 1, i2}, {i1 + 1, i2}, {i1, i2 - 1}, {i1, i2 + 1}};
          for (const MI& m : nb)
            if (m.i1 >= 1 && m.i1 <= c->P.n1 && m.i2 >= 1 && m.i2 <= c->P.n2 && stamp[sub_index(c, m)] == id)
              apart = false;
        }
        ++id;
      }
    S->steps_apart = apart;
  }
  S->subs_host = subs;
  if (c->dense && nrhs < kMatrixRhs && !S->bwd.empty() && c->P.bj_combine == HBJ_BJ_RESTRICTED &&
      !(c->P.bj_compose == HBJ_BJ_RESIDUAL && c->fblocks.size() > 1))
    plan_operator_overlap(c, *S, ent);
  HIPCHK(dalloc(&S->dev, ent.size()));
  HIPCHK(hipMemcpyAsync(S->dev, ent.data(), ent.size() * sizeof(Entry), hipMemcpyHostToDevice, c->st));
  std::vector<FaceTab> eft(ent.size());
  for (size_t q = 0; q < ent.size(); ++q) eft[q] = c->ft_host[ent[q].s];
  HIPCHK(dalloc(&S->eft, eft.size()));
  HIPCHK(hipMemcpyAsync(S->eft, eft.data(), eft.size() * sizeof(FaceTab), hipMemcpyHostToDevice, c->st));
  HIPCHK(dalloc(&S->subs, subs.size()));
  HIPCHK(hipMemcpyAsync(S->subs, subs.data(), subs.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  std::vector<int2> tiles;
  S->all_tile_first = 0;
  append_tiles(ent, S->all_first, S->all_count, tiles);
  S->all_tile_count = (int)tiles.size();
  for (auto* v : {&S->fwd, &S->bwd})
    for (Step& st : *v) {
      st.tile_first = tiles.size();
      append_tiles(ent, st.first, st.count, tiles);
      st.tile_count = (int)(tiles.size() - st.tile_first);
    }
  // small sweep steps of the dense operators take their tables by value (li: row-block list)
  auto by_value = [&](Step& st, int li) {
    const int nrb = c->rbl_n[li];
    if (st.count == 0 || st.count > kStepArgMax || nrb > kStepArgRb) return;
    StepArgs a{};
    for (int q = 0; q < st.count; ++q) {
      a.e[q] = ent[st.first + q];
      a.f[q] = eft[st.first + q];
    }
    for (int q = 0; q < nrb; ++q) a.rb[q] = c->rbl_host[c->rbl_off[li] + q];
    st.sarg = (int)S->sargs.size();
    S->sargs.push_back(a);
  };
  if (!c->rbl_host.empty()) {
    for (Step& st : S->fwd) by_value(st, 0);
    for (Step& st : S->bwd) by_value(st, 1);
  }
  HIPCHK(dalloc(&S->tiles, tiles.size()));
  HIPCHK(hipMemcpyAsync(S->tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  *out = S.get();
  c->sched[nrhs] = std::move(S);
  return HBJ_OK;
}

// The backward solves' window: the kvb rows of U above a column block, then the block.  kvb = kv =
// kl + ku in general; ku when no subdomain's factorisation interchanged rows (U then has ku
// superdiagonals and the window's other rows would only carry zeros).
void set_backward_window(hbj_ctx* c, int kvb) {
  SolveLayout& L = c->L;
  L.wb = L.nb + kvb;
  L.mb_per_sub = (size_t)L.nblk * L.nb * L.wb;
  solve_column_groups(L.wf, L.wb, &L.cgf, &L.cgb);
}

int ensure_ybuf(hbj_ctx* c, size_t entries, size_t elem_bytes) {
  const size_t need = (entries + 1) * (size_t)c->L.nblk * c->L.nb * elem_bytes;  // one spare entry (MFMA solves)
  if (need <= c->ybuf_bytes) return HBJ_OK;
  dfree(c->ybuf);
  c->ybuf = nullptr;
  c->ybuf_bytes = 0;
  if (hipMalloc(&c->ybuf, need) != hipSuccess) return fail(HBJ_ENOMEM, "workspace allocation failed");
  c->ybuf_bytes = need;
  return HBJ_OK;
}

int ensure_loc64(hbj_ctx* c, size_t entries) {
  if (entries <= c->loc64_entries) return HBJ_OK;
  dfree(c->rhs64);
  dfree(c->x64);
  dfree(c->r64);
  c->rhs64 = c->x64 = c->r64 = nullptr;
  c->loc64_entries = 0;
  const size_t n = entries * (size_t)c->g.nloc;
  if (dalloc(&c->rhs64, n) != hipSuccess || dalloc(&c->x64, n) != hipSuccess || dalloc(&c->r64, n) != hipSuccess)
    return fail(HBJ_ENOMEM, "local workspace allocation failed");
  c->loc64_entries = entries;
  return HBJ_OK;
}

int ensure_pc(hbj_ctx* c, size_t ncol) {
  if (ncol <= c->pc_cols) return HBJ_OK;
  dfree(c->pc_y);
  dfree(c->pc_t);
  c->pc_y = c->pc_t = nullptr;
  c->pc_cols = 0;
  const size_t n = ncol * (size_t)c->g.nif;
  if (dalloc(&c->pc_y, n) != hipSuccess || dalloc(&c->pc_t, n) != hipSuccess)
    return fail(HBJ_ENOMEM, "preconditioner workspace allocation failed");
  c->pc_cols = ncol;
  return HBJ_OK;
}

// ---------------------------------------------------------------------------
// profiling: HIP events around a launch group on the context stream
// ---------------------------------------------------------------------------
struct ProfScope {
  hbj_ctx* c;
  int kclass;
  double bytes, flops;
  bool on;  // false: a launch of the autotuner, not counted (the events are the autotuner's)
  ProfScope(hbj_ctx* c_, int k, double b, double f, bool on_ = true) : c(c_), kclass(k), bytes(b), flops(f), on(on_) {
    if (c->prof && on) (void)hipEventRecord(c->ev0, c->st);
  }
  ~ProfScope() {
    if (!c->prof || !on) return;
    (void)hipEventRecord(c->ev1, c->st);
    (void)hipEventSynchronize(c->ev1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    c->ks[kclass].launches += 1;
    c->ks[kclass].ms += ms;
    c->ks[kclass].bytes += bytes;
    c->ks[kclass].flops += flops;
  }
};

// algorithmic bytes of one local solve: factor entries of the band (n_loc (2 kl + ku + 1)),
// the pivot vector, and the solution vector written
double fwd_bytes(const hbj_ctx* c, size_t elem) { return (double)c->g.nloc * c->g.kl * elem + 4.0 * c->g.nloc; }
double bwd_bytes(const hbj_ctx* c, size_t elem) { return (double)c->g.nloc * (solve_kvb(c->L) + 1) * elem; }

// ---------------------------------------------------------------------------
// batched local solves
// ---------------------------------------------------------------------------
// without timing, batches with at least this many entries per tile on average run the MFMA solves
constexpr int kMmMinPerTile = 8;

// runs of a split solve: np runs of bpp column blocks, every run nonempty (np >= 2)
PartLayout part_layout(const hbj_ctx* c) {
  const int nblk = c->L.nblk;
  int np = std::max(2, std::min(c->part_np, nblk));
  int bpp = (nblk + np - 1) / np;
  np = (nblk + bpp - 1) / bpp;
  PartLayout pl{};
  pl.np = np;
  pl.bpp = bpp;
  pl.ns = solve_kvb(c->L);
  return pl;
}

bool part_ok(const hbj_ctx* c) { return c->L.nblk >= 2 && part_fits(c->g, c->L); }

// the split solves' transfer matrices are formed for this factorisation and run count
bool part_ready(const hbj_ctx* c, size_t real_bytes) {
  const int pi = real_bytes == 8 ? 0 : 1;
  const PartLayout pl = part_layout(c);
  return pl.np <= 2 || (c->phi_epoch[pi] == c->graph_epoch && c->phi_np[pi] == pl.np);
}

// workspace of a split-solve batch of nent entries and, once per factorisation, the transfer
// matrices of the runs (formed on the context stream, ahead of the batch)
template <typename R>
hipError_t ensure_part(hbj_ctx* c, int nent, const typename Cplx<R>::T* mf, const typename Cplx<R>::T* mb) {
  typedef typename Cplx<R>::T C;
  const PartLayout pl = part_layout(c);
  const size_t ylen = (size_t)c->L.nblk * c->L.nb;
  auto grow = [](void** p, size_t* have, size_t need) -> hipError_t {
    if (need <= *have) return hipSuccess;
    dfree(*p);
    *p = nullptr;
    *have = 0;
    hipError_t e = hipMalloc(p, need);
    if (e == hipSuccess) *have = need;
    return e;
  };
  hipError_t e = grow(&c->part_y2, &c->part_y2_bytes, (size_t)nent * ylen * sizeof(C));
  if (e == hipSuccess) e = grow(&c->part_st, &c->part_st_bytes, 2 * (size_t)nent * pl.np * pl.ns * sizeof(C));
  if (e == hipSuccess && !c->part_err) {
    e = hipMalloc((void**)&c->part_err, sizeof(int32_t));
    if (e == hipSuccess) e = launch_fill_zero(c->part_err, sizeof(int32_t), c->st);
  }
  const int nctr = part_chain_counters(nent, pl.np);
  if (e == hipSuccess && nctr > c->part_nctr) {  // both regions zero, for the next two launches
    dfree(c->part_ctr);
    c->part_ctr = nullptr;
    c->part_nctr = 0;
    e = hipMalloc((void**)&c->part_ctr, 2 * (size_t)nctr * sizeof(int32_t));
    if (e == hipSuccess) e = launch_fill_zero(c->part_ctr, 2 * (size_t)nctr * sizeof(int32_t), c->st);
    if (e == hipSuccess) {
      c->part_nctr = nctr;
      c->part_parity = 0;
    }
  }
  if (e != hipSuccess || part_ready(c, sizeof(R))) return e;
  const int pi = sizeof(R) == 8 ? 0 : 1;
  const size_t kl = c->g.kl, kv = solve_kvb(c->L), nf = (size_t)c->ndom * (pl.np - 2) * kl * kl;
  e = grow(&c->phi[pi], &c->phi_bytes[pi], (nf + (size_t)c->ndom * (pl.np - 2) * kv * kv) * sizeof(C));
  if (e == hipSuccess)
    e = launch_part_phi<R>(c->g, c->L, pl, mf, c->pf, c->pflag, mb, (C*)c->phi[pi], (C*)c->phi[pi] + nf, c->ndom,
                           c->st);
  if (e != hipSuccess) return e;
  c->phi_epoch[pi] = c->graph_epoch;
  c->phi_np[pi] = pl.np;
  return hipSuccess;
}

// the forward and backward solves of a batch in launch shape `shape` into the solve buffer
template <typename R>
hipError_t solve_pair_shape(hbj_ctx* c, int shape, const Entry* ent, int nent, const int2* tiles, int ntiles,
                            const SolveIO& io, const typename Cplx<R>::T* mf, const typename Cplx<R>::T* mb,
                            bool prof) {
  typedef typename Cplx<R>::T C;
  const bool mm = shape == kShapeMfma;
  const double nread = mm ? (double)ntiles : (double)nent;
  C* sink = (C*)c->ybuf + (size_t)nent * c->L.nblk * c->L.nb;  // the solve buffer holds one spare entry
  hipError_t e;
  if (shape == kShapePart) {
    e = ensure_part<R>(c, nent, mf, mb);
    if (e != hipSuccess) return e;
    const PartLayout pl = part_layout(c);
    const int pi = sizeof(R) == 8 ? 0 : 1;
    const size_t nf = (size_t)c->ndom * (pl.np - 2) * c->g.kl * c->g.kl;
    const C* phi_f = (const C*)c->phi[pi];
    const C* phi_b = phi_f ? phi_f + nf : nullptr;
    C* sig = (C*)c->part_st;
    C* tt = sig + (size_t)nent * pl.np * pl.ns;
    PartWait pw{c->part_ctr, c->part_nctr, c->part_parity, c->part_err, c->df_spin};
    {
      ProfScope ps(c, HBJ_K_FWD, nread * fwd_bytes(c, sizeof(C)), nent * 8.0 * c->g.nloc * c->g.kl, prof);
      e = launch_fwd_part<R>(c->g, c->L, pl, ent, nent, c->ft, c->coef, mf, c->pf, c->pflag, phi_f, io, (C*)c->ybuf,
                             (C*)c->part_y2, sig, tt, pw, c->st);
    }
    c->part_parity = pw.parity;
    if (e != hipSuccess) return e;
    ProfScope ps(c, HBJ_K_BWD, nread * bwd_bytes(c, sizeof(C)), nent * 8.0 * c->g.nloc * (solve_kvb(c->L) + 1), prof);
    e = launch_bwd_part<R>(c->g, c->L, pl, ent, nent, c->ft, c->coef, mb, phi_b, io, (const C*)c->part_y2,
                           (C*)c->ybuf, sig, tt, pw, c->st);
    c->part_parity = pw.parity;
    return e;
  }
  {
    ProfScope ps(c, HBJ_K_FWD, nread * fwd_bytes(c, sizeof(C)), nent * 8.0 * c->g.nloc * c->g.kl, prof);
    e = mm ? launch_fwd_mm<R>(c->g, c->L, ent, tiles, ntiles, c->ft, c->coef, mf, c->pf, c->pflag, c->interchanges,
                              io, (C*)c->ybuf, sink, c->st)
           : launch_fwd<R>(c->g, c->L, ent, nent, c->ft, c->coef, mf, c->pf, c->pflag, io, (C*)c->ybuf, c->st, shape);
  }
  if (e != hipSuccess) return e;
  {
    ProfScope ps(c, HBJ_K_BWD, nread * bwd_bytes(c, sizeof(C)), nent * 8.0 * c->g.nloc * (solve_kvb(c->L) + 1), prof);
    e = mm ? launch_bwd_mm<R>(c->g, c->L, ent, tiles, ntiles, c->ft, c->coef, mb, io, (C*)c->ybuf, sink, c->st)
           : launch_bwd<R>(c->g, c->L, ent, nent, c->ft, c->coef, mb, io, (C*)c->ybuf, c->st, shape);
  }
  return e;
}

// average right-hand sides per 16-wide tile of a batch (rounded up)
int per_tile(int nent, int ntiles) { return ntiles > 0 ? (nent + ntiles - 1) / ntiles : 0; }

// cache key of a batch class: device, precision, subdomain and band, backward window, interchanges,
// number of solves (next power of two), average right-hand sides per subdomain tile (1, 2, 4, 8, 16),
// and whether the batch may skip solves with zero right-hand sides (the lifting and reconstruction of
// a localised source: their cost depends on the data, so they do not decide for the operator's batches)
std::string solve_class_key(const hbj_ctx* c, size_t elem, int nent, int ntiles, bool mm_ok, bool skips) {
  int n2 = 1;
  while (n2 < nent) n2 *= 2;
  const int per = mm_ok ? per_tile(nent, ntiles) : 1;
  const int pb = per >= 16 ? 16 : per >= 8 ? 8 : per >= 4 ? 4 : per >= 2 ? 2 : 1;
  char buf[160];
  std::snprintf(buf, sizeof buf, "solve|%s|%s|%dx%d|kl%d|ku%d|wb%d|p%d|n%d|r%d|%s|z%d|s%d|np%d", c->arch.c_str(),
                elem == 16 ? "c128" : "c64", c->g.snx, c->g.sny, c->g.kl, c->g.ku, c->L.wb, c->interchanges ? 1 : 0, n2,
                pb, mm_ok ? "mm" : "wg", skips ? 1 : 0, kSolveShapes, part_layout(c).np);
  return std::string(buf);
}

bool tuning_enabled(const hbj_ctx* c) {
  const char* env = std::getenv("HBJ_TUNE");
  if (env && std::strcmp(env, "0") == 0) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  return true;
}

// autotuner of the banded solve batches: every candidate shape runs on this batch's own data
// with the outputs switched off (only the solve buffer is written), once to warm up and to drop
// candidates at more than twice the best time, then three rounds in turns; the fastest wins
template <typename R>
int time_solve_shapes(hbj_ctx* c, const Entry* ent, int nent, const int2* tiles, int ntiles, const SolveIO& io,
                      const typename Cplx<R>::T* mf, const typename Cplx<R>::T* mb, bool mm_ok,
                      hbj_ctx::SolveChoice& ch) {
  HIPCHK(hipDeviceSynchronize());  // the side stream may still run a reconstruction's source part
  SolveIO tio = io;
  tio.u = nullptr;
  tio.x64 = nullptr;
  tio.tr_dst = nullptr;
  bool alive[kSolveShapes];
  float first[kSolveShapes] = {}, tot[kSolveShapes] = {};
  // the split solves are candidates for batches of one or two right-hand sides per subdomain (many right-hand
  // sides per subdomain fill the device, on MFMA or with one workgroup per solve; their transfer matrices
  // would only cost memory and time)
  const bool split_ok = part_ok(c) && (!tiles || ntiles <= 0 || per_tile(nent, ntiles) <= 2);
  for (int v = 0; v < kSolveShapes; ++v) alive[v] = (v != kShapeMfma || mm_ok) && (v != kShapePart || split_ok);
  if (alive[kShapePart]) HIPCHK(ensure_part<R>(c, nent, mf, mb));  // formed once, outside the timings
  auto timed = [&](int v, float* ms) -> hipError_t {
    hipError_t e = hipEventRecord(c->ev0, c->st);
    if (e == hipSuccess) e = solve_pair_shape<R>(c, v, ent, nent, tiles, ntiles, tio, mf, mb, false);
    if (e == hipSuccess) e = hipEventRecord(c->ev1, c->st);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, c->ev0, c->ev1);
    return e;
  };
  float best = 1e30f;
  for (int v = 0; v < kSolveShapes; ++v) {
    if (!alive[v]) continue;
    HIPCHK(timed(v, &first[v]));
    best = std::min(best, first[v]);
  }
  for (int v = 0; v < kSolveShapes; ++v)
    if (alive[v] && first[v] > 2.0f * best) alive[v] = false;
  for (int rep = 0; rep < 3; ++rep)
    for (int v = 0; v < kSolveShapes; ++v) {
      if (!alive[v]) continue;
      float ms = 0.f;
      HIPCHK(timed(v, &ms));
      tot[v] += ms;
    }
  int pick = -1;
  for (int v = 0; v < kSolveShapes; ++v) {
    ch.us[v] = alive[v] ? tot[v] / 3.0f * 1e3f : first[v] * 1e3f;
    if (alive[v] && (pick < 0 || tot[v] < tot[pick])) pick = v;
  }
  ch.shape = pick < 0 ? 0 : pick;
  return HBJ_OK;
}

// forward and backward solves of a batch into the solve buffer, in the launch shape chosen for
// the batch's class: fixed by hbj_set_solve_tuning, chosen earlier in this process, read from
// the tuning cache file, or timed now
template <typename R>
int launch_solve_pair(hbj_ctx* c, const Entry* ent, int nent, const int2* tiles, int ntiles, const SolveIO& io,
                      const typename Cplx<R>::T* mf, const typename Cplx<R>::T* mb) {
  typedef typename Cplx<R>::T C;
  const bool mm_ok = c->msolve == HBJ_MSOLVE_MFMA && tiles && ntiles > 0 && trisolve_mm_fits(c->L, sizeof(C));
  int shape;
  if (c->solve_shape_fixed >= 0) {
    shape = c->solve_shape_fixed;
    if ((shape == kShapeMfma && !mm_ok) || (shape == kShapePart && !part_ok(c))) shape = 0;
  } else {
    const std::string key = solve_class_key(c, sizeof(C), nent, ntiles, mm_ok, io.nz != nullptr);
    auto it = c->solve_choice.find(key);
    if (it != c->solve_choice.end()) {
      shape = it->second.shape;
    } else {
      hbj_ctx::SolveChoice ch;
      int v = -1;
      if (tune_cache_get(key, &v) && v >= 0 && v < kSolveShapes && (v != kShapeMfma || mm_ok) &&
          (v != kShapePart || part_ok(c))) {
        ch.shape = v;
      } else if (tuning_enabled(c)) {
        int rc = time_solve_shapes<R>(c, ent, nent, tiles, ntiles, io, mf, mb, mm_ok, ch);
        if (rc) return rc;
        tune_cache_put(key, ch.shape, ch.us, kSolveShapes);  // a file that cannot be written only loses the cache
      } else {
        ch.shape = (mm_ok && per_tile(nent, ntiles) >= kMmMinPerTile) ? kShapeMfma : 0;
      }
      c->solve_choice[key] = ch;
      shape = ch.shape;
    }
  }
  if (shape == kShapePart && !tuning_enabled(c) && !part_ready(c, sizeof(R))) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) shape = 0;
  }
  HIPCHK(solve_pair_shape<R>(c, shape, ent, nent, tiles, ntiles, io, mf, mb, true));
  return HBJ_OK;
}

template <typename R>
int run_solves(hbj_ctx* c, const Entry* ent, int nent, const SolveIO& io_in, const int2* tiles = nullptr,
               int ntiles = 0) {
  typedef typename Cplx<R>::T C;
  if (nent == 0) return HBJ_OK;
  int rc = ensure_ybuf(c, nent, sizeof(C));
  if (rc) return rc;
  // second-order transmission: the data sent across a face need the field along the whole face,
  // so the solves write the local fields and the traces follow from them in a second kernel
  SolveIO io = io_in;
  double2* field = nullptr;
  if (io_in.tr_dst && c->P.transmission == 2) {
    field = io_in.x64;
    if (!field) {
      if ((size_t)nent > c->xtr_entries) {
        dfree(c->xtr);
        c->xtr = nullptr;
        c->xtr_entries = 0;
        if (dalloc(&c->xtr, (size_t)nent * c->g.nloc)) return fail(HBJ_ENOMEM, "trace workspace allocation failed");
        c->xtr_entries = nent;
      }
      field = c->xtr;
    }
    io.tr_dst = nullptr;
    io.x64 = field;
  }
  const C* mf;
  const C* mb;
  if constexpr (sizeof(R) == 8) {
    mf = c->mf64;
    mb = c->mb64;
  } else {
    mf = c->mf32;
    mb = c->mb32;
  }
  rc = launch_solve_pair<R>(c, ent, nent, tiles, ntiles, io, mf, mb);
  if (rc) return rc;
  if (field) {
    SolveIO tio = io_in;
    tio.u = nullptr;
    tio.x64 = nullptr;
    HIPCHK(launch_emit_traces(c->g, ent, nent, c->ft, c->band, tio, field, c->st));
  }
  c->local_solves += nent;
  return HBJ_OK;
}

// FP64 local solves of a batch on the side stream (own workspace, not profiled)
int run_solves_side(hbj_ctx* c, const Entry* ent, int nent, const SolveIO& io) {
  if (nent == 0) return HBJ_OK;
  const size_t need = (size_t)nent * c->L.nblk * c->L.nb * sizeof(double2);
  if (need > c->ybuf_side_bytes) {
    dfree(c->ybuf_side);
    c->ybuf_side = nullptr;
    c->ybuf_side_bytes = 0;
    if (hipMalloc(&c->ybuf_side, need) != hipSuccess) return fail(HBJ_ENOMEM, "workspace allocation failed");
    c->ybuf_side_bytes = need;
  }
  HIPCHK((launch_fwd<double>(c->g, c->L, ent, nent, c->ft, c->coef, c->mf64, c->pf, c->pflag, io,
                             (double2*)c->ybuf_side, c->side)));
  HIPCHK((launch_bwd<double>(c->g, c->L, ent, nent, c->ft, c->coef, c->mb64, io, (double2*)c->ybuf_side, c->side)));
  c->local_solves += nent;
  return HBJ_OK;
}

// batched application of the dense scattering operators (complex128 or complex64 storage)

int run_dense(hbj_ctx* c, const Entry* ent, const FaceTab* eft, int nent, int mask, const SolveIO& io, bool c64,
              double elems,
              const int32_t* subs = nullptr, int nsub = 0, int nrhs = 1, int src = 0, const StepArgs* sa = nullptr,
              const void* Gpre = nullptr) {
  if (nent == 0) return HBJ_OK;
  if (subs && nrhs >= kMatrixRhs) {
    const int rpad = (nrhs + 15) / 16 * 16;
    const size_t need = (size_t)nsub * local_if_len(c->g) * rpad;
    if (need > c->Gbuf_cap) {
      dfree(c->Gbuf);
      c->Gbuf = nullptr;
      c->Gbuf_cap = 0;
      if (dalloc(&c->Gbuf, need)) return fail(HBJ_ENOMEM, "operator workspace allocation failed");
      c->Gbuf_cap = need;
    }
    // per subdomain the operator is read once for all right-hand sides
    const double tbytes = elems / nrhs * (c64 ? 8.0 : 16.0);
    const double2* gin = src ? io.g_b : io.g_a;
    const int slot = (c64 ? 2 : 0) + (mask == 0xF ? 1 : 0);
    // variants 0-2 and 6-8 gather the incoming data into tiles first (in complex64 for the
    // complex64 products, which round every operand to float anyway); the others read them from
    // gin directly
    // (Gpre: the tiles are already gathered, by a chained pass)
    auto launch = [&](int v, const SolveIO& lio) -> hipError_t {
      if (mm_variant_gathered(v) && !Gpre) {
        const hipError_t e =
            c64 ? launch_gather_incoming(c->g, subs, nsub, c->ft, gin, nrhs, rpad, (float2*)c->Gbuf, c->st)
                : launch_gather_incoming(c->g, subs, nsub, c->ft, gin, nrhs, rpad, c->Gbuf, c->st);
        if (e != hipSuccess) return e;
      }
      const void* G = Gpre ? Gpre : (const void*)c->Gbuf;
      return c64 ? launch_scatter_mm<float2>(c->g, subs, nsub, mask, c->ft, c->T32, gin, (const float2*)G, nrhs,
                                             rpad, lio, c->st, v)
                 : launch_scatter_mm<double2>(c->g, subs, nsub, mask, c->ft, c->T64, gin, (const double2*)G, nrhs,
                                              rpad, lio, c->st, v);
    };
    // cache key of this launch kind: device, precision, operator or steps, checkerboard, subdomain,
    // padded right-hand sides (by powers of two)
    char mkey[128];
    {
      int r2 = 16;
      while (r2 < rpad && r2 < 128) r2 *= 2;
      std::snprintf(mkey, sizeof mkey, "mm|%s|%s|%s|%dx%d|%dx%d|r%d", c->arch.c_str(), c64 ? "c64" : "c128",
                    mask == 0xF ? "op" : "steps", c->g.n1, c->g.n2, c->g.snx, c->g.sny, r2);
    }
    if (c->mm_variant[slot] < 0) {
      int v = -1;
      if (!(tune_cache_get(mkey, &v) && v >= 0 && v < kMmVariants) && !tuning_enabled(c))
        v = mask == 0xF ? 7 : 15;  // no timing allowed: the usual winners on gfx950 (see hbj_get_tuning)
      if (v >= 0) {
        c->mm_variant[slot] = v;
        for (int q = 0; q < kMmVariants; ++q) c->mm_us[slot][q] = 0.f;
      }
    }
    if (c->mm_variant[slot] < 0) {
      // autotuner: time every variant on this very launch, writing into scratch, keep the fastest
      // (after the device is idle: the source part of a reconstruction may still run on the second
      // stream, and the variants timed beside it would look slower)
      HIPCHK(hipDeviceSynchronize());
      double2* scratch = nullptr;
      if (dalloc(&scratch, (size_t)nrhs * c->g.nif)) return fail(HBJ_ENOMEM, "tuning workspace allocation failed");
      SolveIO tio = io;
      tio.tr_dst = scratch;
      tio.tr_base = nullptr;
      tio.cmap = nullptr;  // the next tile is written by the launch proper
      // the variants take turns (three rounds after a warm-up round), so that each one is timed after
      // another has streamed its data, as in a solve, rather than on caches it has just filled itself
      // (the warm-up round is timed too: a variant at more than twice the best time there drops out)
      hipError_t he = hipSuccess;
      float tot[kMmVariants] = {}, first[kMmVariants] = {};
      bool alive[kMmVariants];
      auto timed = [&](int v, float* ms) -> hipError_t {
        hipError_t e = hipEventRecord(c->ev0, c->st);
        if (e == hipSuccess) e = launch(v, tio);
        if (e == hipSuccess) e = hipEventRecord(c->ev1, c->st);
        if (e == hipSuccess) e = hipEventSynchronize(c->ev1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, c->ev0, c->ev1);
        return e;
      };
      float fbest = 1e30f;
      for (int v = 0; v < kMmVariants && he == hipSuccess; ++v) {
        he = timed(v, &first[v]);
        fbest = std::min(fbest, first[v]);
      }
      for (int v = 0; v < kMmVariants; ++v) alive[v] = first[v] <= 2.0f * fbest;
      for (int rep = 0; rep < 3 && he == hipSuccess; ++rep)
        for (int v = 0; v < kMmVariants && he == hipSuccess; ++v) {
          if (!alive[v]) continue;
          float ms = 0.f;
          he = timed(v, &ms);
          tot[v] += ms;
        }
      int best = -1;
      for (int v = 0; v < kMmVariants; ++v) {
        c->mm_us[slot][v] = (alive[v] ? tot[v] / 3.0f : first[v]) * 1e3f;
        if (alive[v] && (best < 0 || tot[v] < tot[best])) best = v;
      }
      (void)hipStreamSynchronize(c->st);
      dfree(scratch);
      if (he != hipSuccess) return fail(HBJ_EHIP, hipGetErrorString(he));
      c->mm_variant[slot] = best < 0 ? 0 : best;
      tune_cache_put(mkey, c->mm_variant[slot], c->mm_us[slot], kMmVariants);  // a write failure only loses the cache
    }
    ProfScope ps(c, mask == 0xF ? HBJ_K_OPERATOR : HBJ_K_SCATTER, tbytes, elems * 8.0);
    HIPCHK(launch(c->mm_variant[slot], io));
    return HBJ_OK;
  }
  const int li = mask == kMaskFwd ? 0 : mask == kMaskBwd ? 1 : 2;
  const int32_t* rbl = c->rbl + c->rbl_off[li];
  // profiling: the dispatch's own start and stop times (no event packets around the launch)
  hipEvent_t t0 = c->prof ? c->ev0 : nullptr, t1 = c->prof ? c->ev1 : nullptr;
  if (c64)
    HIPCHK(launch_scatter_apply<float2>(c->g, ent, nent, mask, rbl, c->rbl_n[li], eft, c->T32, io, c->st, t0, t1, sa));
  else
    HIPCHK(launch_scatter_apply<double2>(c->g, ent, nent, mask, rbl, c->rbl_n[li], eft, c->T64, io, c->st, t0, t1, sa));
  if (c->prof) {
    HIPCHK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    hbj_kernel_stat& k = c->ks[mask == 0xF ? HBJ_K_OPERATOR : HBJ_K_SCATTER];
    k.launches += 1;
    k.ms += ms;
    k.bytes += elems * (c64 ? 8.0 : 16.0);
    k.flops += elems * 8.0;
  }
  return HBJ_OK;
}

// ---------------------------------------------------------------------------
// dataflow sweeps (dense form, few right-hand sides)
// ---------------------------------------------------------------------------
// row blocks of subdomain s holding a row of a face in mask that writes an outgoing datum (or,
// with copy, passes an incoming datum through)
std::vector<int> df_row_blocks(const hbj_ctx* c, int s, int mask, bool copy) {
  const int L = local_if_len(c->g);
  const FaceTab& F = c->ft_host[s];
  std::vector<int> out;
  for (int rb = 0; rb * kTR < L; ++rb) {
    bool use = false;
    for (int row = rb * kTR; row < std::min(L, rb * kTR + kTR); ++row) {
      int f, e;
      local_if_face(c->g, row, &f, &e);
      if (((mask >> f) & 1) && (F.out_off[f] >= 0 || (copy && F.in_off[f] >= 0))) use = true;
    }
    if (use) out.push_back(rb);
  }
  return out;
}

// Task lists in topological order.  Stage 0 = forward pass, 1 = backward pass, 2 = operator.
// Dependencies (data written by another task of the same launch):
//  forward, after the first step of an interval: the forward tasks of the W and S neighbours
//    (they write this subdomain's W and S incoming blocks);
//  backward, after the first step: the backward tasks of the E and N neighbours; in a launch
//    that also runs the forward pass, the forward tasks of the subdomain and of its W and S
//    neighbours (they write or pass through every block the backward task reads);
//  operator after the backward pass: the backward tasks of the subdomain and of its E and N
//    neighbours.
int build_df(hbj_ctx* c, Schedule* S, int kind) {
  Schedule::DfPlan& P = S->df[kind];
  if (P.built) return HBJ_OK;
  const int nd = c->ndom, nrhs = S->nrhs, n1 = c->P.n1, n2 = c->P.n2;
  const bool has[3] = {kind == DF_FWD || kind == DF_PC || kind == DF_PC_OP,
                       kind == DF_BWD || kind == DF_PC || kind == DF_PC_OP, kind == DF_PC_OP || kind == DF_OP};
  const int smask[3] = {kMaskFwd, kMaskBwd, 0xF};
  const int scopy[3] = {1, 1, 0};
  // (subdomain, first) per step of each stage, in sweep order
  std::vector<std::vector<std::pair<int, int>>> order[3];
  if (has[0] || has[1]) {
    int nsteps = 0;
    for (auto& b : c->fblocks) nsteps = std::max(nsteps, b.second - b.first);
    for (int t = 1; t <= nsteps; ++t) {
      std::vector<std::pair<int, int>> step;
      for (auto& b : c->fblocks) {
        if (b.first + t > b.second) continue;
        for (int s : antidiag_subdomains(c, b.first + t - 1)) step.push_back({s, t == 1});
      }
      order[0].push_back(step);
    }
    nsteps = 0;
    for (auto& b : c->bblocks) nsteps = std::max(nsteps, b.second - b.first);
    for (int t = 1; t <= nsteps; ++t) {
      std::vector<std::pair<int, int>> step;
      for (auto& b : c->bblocks) {
        if (b.second - t < b.first) continue;
        for (int s : antidiag_subdomains(c, b.second - t + 1)) step.push_back({s, t == 1});
      }
      order[1].push_back(step);
    }
  }
  std::vector<std::pair<int, int>> all;
  for (int s = 0; s < nd; ++s) all.push_back({s, 1});
  order[2].push_back(all);
  std::vector<std::vector<int>> rbs[3];
  std::vector<int> ntk[3];
  for (int st = 0; st < 3; ++st) {
    rbs[st].assign(nd, {});
    ntk[st].assign(nd, 0);
    if (!has[st]) continue;
    for (auto& step : order[st])
      for (auto& it : step) {
        rbs[st][it.first] = df_row_blocks(c, it.first, smask[st], scopy[st]);
        ntk[st][it.first] = (int)rbs[st][it.first].size();
      }
  }
  auto slot = [&](int st, int s, int r) { return (st * nd + s) * nrhs + r; };
  auto nb = [&](int s, int f) {  // neighbour through face f (W, E, S, N) or -1
    const int i1 = s % n1, i2 = s / n1;
    if (f == FACE_W) return i1 > 0 ? s - 1 : -1;
    if (f == FACE_E) return i1 < n1 - 1 ? s + 1 : -1;
    if (f == FACE_S) return i2 > 0 ? s - n1 : -1;
    return i2 < n2 - 1 ? s + n1 : -1;
  };
  std::vector<DfTask> tasks;
  double tbytes = 0, flops = 0;
  // operator bytes of one task: complex64 in the preconditioner of the mixed form, complex128 else
  const double row_elems = (double)local_if_len(c->g) * kTR;
  const double pc_eb = c->P.precision == HBJ_MIXED ? 8.0 : 16.0;
  for (int st = 0; st < 3; ++st) {
    if (!has[st]) continue;
    for (auto& step : order[st])
      for (auto& it : step) {
        const int s = it.first, first = it.second;
        for (int r = 0; r < nrhs; ++r) {
          std::vector<std::pair<int, int>> deps;
          auto dep_on = [&](int dst, int q) {
            if (q >= 0 && ntk[dst][q] > 0) deps.push_back({slot(dst, q, r), ntk[dst][q]});
          };
          if (st == 0 && !first) {
            dep_on(0, nb(s, FACE_W));
            dep_on(0, nb(s, FACE_S));
          }
          if (st == 1) {
            if (!first) {
              dep_on(1, nb(s, FACE_E));
              dep_on(1, nb(s, FACE_N));
            }
            if (has[0]) {
              dep_on(0, s);
              dep_on(0, nb(s, FACE_W));
              dep_on(0, nb(s, FACE_S));
            }
          }
          if (st == 2 && has[1]) {
            dep_on(1, s);
            dep_on(1, nb(s, FACE_E));
            dep_on(1, nb(s, FACE_N));
          }
          if (deps.size() > (size_t)kDfMaxDeps) return fail(HBJ_EINVAL, "dataflow plan: too many dependencies");
          for (int rb : rbs[st][s]) {
            DfTask t{};
            t.stage = st;
            t.s = s;
            t.rhs = r;
            t.rb = rb;
            t.first = first;
            t.slot = slot(st, s, r);
            t.ndep = (int)deps.size();
            for (size_t d = 0; d < deps.size(); ++d) {
              t.dep[d] = deps[d].first;
              t.need[d] = deps[d].second;
            }
            tasks.push_back(t);
            tbytes += row_elems * (st == 2 ? 16.0 : pc_eb);
            flops += row_elems * 8.0;
          }
        }
      }
  }
  // every wait must be on tasks with smaller tickets, for exactly the number of tasks behind
  // the counter: checked here so that a plan that could stall is never launched
  {
    std::vector<int> last(3 * (size_t)nd * nrhs, -1), count(3 * (size_t)nd * nrhs, 0);
    for (size_t i = 0; i < tasks.size(); ++i) {
      last[tasks[i].slot] = (int)i;
      count[tasks[i].slot] += 1;
    }
    for (size_t i = 0; i < tasks.size(); ++i)
      for (int d = 0; d < tasks[i].ndep; ++d) {
        const int q = tasks[i].dep[d];
        if (last[q] < 0 || last[q] >= (int)i || count[q] != tasks[i].need[d])
          return fail(HBJ_EINVAL, "dataflow plan: a task would wait on a later or miscounted task");
      }
  }
  if (!S->df_ctr) {
    S->df_nctr = 1 + 3 * nd * nrhs;
    if (dalloc(&S->df_ctr, 2 * (size_t)S->df_nctr)) return fail(HBJ_ENOMEM, "dataflow counter allocation failed");
    HIPCHK(launch_fill_zero(S->df_ctr, 2 * (size_t)S->df_nctr * sizeof(int32_t), c->st));
    S->df_parity = 0;
  }
  if (dalloc(&P.dev, tasks.size())) return fail(HBJ_ENOMEM, "dataflow plan allocation failed");
  HIPCHK(hipMemcpyAsync(P.dev, tasks.data(), tasks.size() * sizeof(DfTask), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  P.ntasks = (int)tasks.size();
  P.tbytes = tbytes;
  P.flops = flops;
  P.built = true;
  return HBJ_OK;
}

bool df_enabled(const hbj_ctx* c, const Schedule* S) {
  return c->dense && c->P.sweep_exec == HBJ_SWEEP_DATAFLOW && S->nrhs < kMatrixRhs;
}

DfStage df_stage(const double2* in, const double2* out, double2* dst, const double2* base, double sign, int mask,
                 int copy) {
  DfStage st{};
  st.in = in;
  st.out = out;
  st.dst = dst;
  st.base = base;
  st.sign = sign;
  st.mask = mask;
  st.out_read = (~mask) & 0xF;
  st.copy = copy;
  return st;
}

template <typename C>
int run_df(hbj_ctx* c, Schedule* S, int kind, const DfArgs& A, const C* T) {
  int rc = build_df(c, S, kind);
  if (rc) return rc;
  const Schedule::DfPlan& P = S->df[kind];
  if (P.ntasks == 0) return HBJ_OK;
  int32_t* cur = S->df_ctr + (size_t)S->df_parity * S->df_nctr;
  int32_t* nxt = S->df_ctr + (size_t)(1 - S->df_parity) * S->df_nctr;
  const int grid = std::min(P.ntasks, c->df_grid);
  {
    ProfScope ps(c, HBJ_K_SWEEP, P.tbytes, P.flops);
    HIPCHK(launch_sweep_df<C>(c->g, P.dev, P.ntasks, c->ft, T, A, cur, nxt, S->df_nctr, c->df_err, c->df_spin,
                              c->df_stall, grid, c->st));
  }
  S->df_parity ^= 1;
  return HBJ_OK;
}

// wait failures of earlier chain launches of split solves (synchronises the stream)
int part_check(hbj_ctx* c) {
  if (!c->part_err) return HBJ_OK;
  int32_t e = 0;
  HIPCHK(hipMemcpyAsync(&e, c->part_err, sizeof(e), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (!e) return HBJ_OK;
  HIPCHK(launch_fill_zero(c->part_err, sizeof(int32_t), c->st));
  if (c->part_ctr) HIPCHK(launch_fill_zero(c->part_ctr, 2 * (size_t)c->part_nctr * sizeof(int32_t), c->st));
  c->part_parity = 0;
  HIPCHK(hipStreamSynchronize(c->st));
  return fail(HBJ_EWAIT, "split local solves: a wait of the transfer chain exceeded its poll limit");
}

// dependency-wait failures of earlier dataflow launches and split solves (synchronises the stream)
int df_check(hbj_ctx* c) {
  const int rp = part_check(c);
  if (rp) return rp;
  if (!c->df_err) return HBJ_OK;
  int32_t e = 0;
  HIPCHK(hipMemcpyAsync(&e, c->df_err, sizeof(e), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (!e) return HBJ_OK;
  HIPCHK(launch_fill_zero(c->df_err, sizeof(int32_t), c->st));
  for (auto& kv : c->sched) {
    Schedule* S = kv.second.get();
    if (S->df_ctr) HIPCHK(launch_fill_zero(S->df_ctr, 2 * (size_t)S->df_nctr * sizeof(int32_t), c->st));
    S->df_parity = 0;
  }
  HIPCHK(hipStreamSynchronize(c->st));
  return fail(HBJ_EWAIT, "dataflow sweep: a dependency wait exceeded its poll limit");
}

// The lifting matrices serve few right-hand sides (one matrix-vector product each); many
// right-hand sides keep the batched banded solves, which read each factor once per launch.
bool is_pade(const hbj_ctx* c) { return c->P.transmission == 3; }

bool dense_lift(const hbj_ctx* c, int nrhs) { return c->Wl && (nrhs < kMatrixRhs || is_pade(c)); }

// lifting b = traces of A^{-1} f: subdomains whose source restriction is identically zero
// contribute exactly zero and skip their solves
int run_lifting(hbj_ctx* c, Schedule* S, const double2* f, double2* b, int nrhs) {
  if (is_pade(c) && !c->Wl) return fail(HBJ_ESTATE, "the Pade transmission needs the dense lifting matrices");
  const size_t need = (size_t)nrhs * c->ndom;
  if (need > c->nzf_cap) {
    dfree(c->nzf);
    c->nzf = nullptr;
    c->nzf_cap = 0;
    if (dalloc(&c->nzf, need)) return fail(HBJ_ENOMEM, "flag allocation failed");
    c->nzf_cap = need;
  }
  HIPCHK(launch_source_flags(c->g, f, nrhs, c->nzf, c->st));
  if (dense_lift(c, nrhs)) {
    // dense lifting operators: one matrix-vector product per (subdomain, rhs) with a source
    std::vector<int32_t> nzh(need);
    HIPCHK(hipMemcpyAsync(nzh.data(), c->nzf, need * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const int L = local_if_len(c->g);
    const int nchunk = lift_chunks(c->g, kLiftChunk);
    const size_t per_rhs = (size_t)c->ndom * nchunk * L;
    const int batch = (int)std::max<size_t>(1, std::min<size_t>(nrhs, kLiftPartialElems / per_rhs));
    if ((size_t)batch * per_rhs > c->lpart_cap) {
      dfree(c->lpart);
      c->lpart = nullptr;
      c->lpart_cap = 0;
      if (dalloc(&c->lpart, (size_t)batch * per_rhs)) return fail(HBJ_ENOMEM, "lifting workspace allocation failed");
      c->lpart_cap = (size_t)batch * per_rhs;
    }
    for (int r0 = 0; r0 < nrhs; r0 += batch) {
      const int nb = std::min(batch, nrhs - r0);
      double pairs = 0;
      for (size_t q = (size_t)r0 * c->ndom; q < (size_t)(r0 + nb) * c->ndom; ++q) pairs += nzh[q] != 0;
      ProfScope ps(c, HBJ_K_LIFT, pairs * (double)c->g.nloc * L * 16.0, pairs * 8.0 * c->g.nloc * L);
      if (is_pade(c)) {
        // y = W^T f per chunk, then b = -Sigma G^-T y along each face
        HIPCHK(launch_lift_partials(c->g, c->Wl, f + (size_t)r0 * c->g.nx * c->g.ny, c->nzf + (size_t)r0 * c->ndom,
                                    nb, kLiftChunk, c->lpart, c->st));
        HIPCHK(launch_pade_lift(c->g, c->ft, c->pade_S, c->Ginv, c->nzf + (size_t)r0 * c->ndom, c->lpart, nchunk, nb,
                                b + (size_t)r0 * c->g.nif, c->st));
        continue;
      }
      HIPCHK(launch_lift_dense(c->g, c->ft, c->band, c->Wl, f + (size_t)r0 * c->g.nx * c->g.ny,
                               c->nzf + (size_t)r0 * c->ndom,
                               nb, kLiftChunk, c->lpart, b + (size_t)r0 * c->g.nif, c->st));
    }
    return HBJ_OK;
  }
  SolveIO io{};
  io.f = f;
  io.nz = c->nzf;
  io.tr_dst = b;
  io.tr_sign = 1.0;
  io.tr_reflect = 0;
  return run_solves<double>(c, S->dev + S->all_first, S->all_count, io, S->tiles + S->all_tile_first, S->all_tile_count);
}

// Source part of the reconstruction, u_s = A_s^{-1} f_s (zero where f_s = 0), on the side
// stream once the flags of run_lifting are known; the main stream goes on with GMRES.
int fork_source_part(hbj_ctx* c, Schedule* S, const double2* f, double2* u) {
  if (!c->side) {
    HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(c->ev_fork, c->st));
  HIPCHK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
  SolveIO io{};
  io.f = f;
  io.nz = c->nzf;
  io.nz_skip_out = 1;
  io.u = u;
  int rc = run_solves_side(c, S->dev + S->all_first, S->all_count, io);
  if (rc) return rc;
  HIPCHK(hipEventRecord(c->ev_join, c->side));
  return HBJ_OK;
}

// u = A^{-1}(f + B g) on every subdomain.  Dense form: u holds the source part (from the side
// stream when source_done, else computed here) and the transmission part is one product with
// the lifting matrices per subdomain; banded form: one local solve per subdomain.
int run_reconstruct(hbj_ctx* c, Schedule* S, const double2* f, const double2* g, double2* u, int nrhs,
                    bool source_done) {
  if (is_pade(c) && !c->Wl) return fail(HBJ_ESTATE, "the Pade transmission needs the dense lifting matrices");
  if (c->Wl && c->g.nif > 0 && g) {
    if (source_done) {
      HIPCHK(hipStreamWaitEvent(c->st, c->ev_join, 0));
    } else {
      const size_t need = (size_t)nrhs * c->ndom;
      if (need > c->nzf_cap) {
        dfree(c->nzf);
        c->nzf = nullptr;
        c->nzf_cap = 0;
        if (dalloc(&c->nzf, need)) return fail(HBJ_ENOMEM, "flag allocation failed");
        c->nzf_cap = need;
      }
      HIPCHK(launch_source_flags(c->g, f, nrhs, c->nzf, c->st));
      SolveIO io{};
      io.f = f;
      io.nz = c->nzf;
      io.nz_skip_out = 1;
      io.u = u;
      int rc = run_solves<double>(c, S->dev + S->all_first, S->all_count, io, S->tiles + S->all_tile_first, S->all_tile_count);
      if (rc) return rc;
    }
    if (is_pade(c)) {
      // u holds v = A_b^-1 f (the band factors keep the Robin closure): the transmission part
      // becomes Y G^-1 (J g - C U^T v), handed to the products below as incoming data gt
      // workspace: gt [nrhs][nif], then q [nrhs][ndom][L]
      const size_t nq = (size_t)nrhs * c->ndom * local_if_len(c->g);
      const size_t need = (size_t)nrhs * c->g.nif + nq;
      if (need > c->pade_gt_cap) {
        dfree(c->pade_gt);
        c->pade_gt = nullptr;
        c->pade_gt_cap = 0;
        if (dalloc(&c->pade_gt, need)) return fail(HBJ_ENOMEM, "reconstruction workspace allocation failed");
        c->pade_gt_cap = need;
      }
      HIPCHK(launch_pade_recon_prep(c->g, c->ft, c->coef, c->pade_J, c->pade_C, c->Ginv, g, c->nzf, u, nrhs,
                                    c->pade_gt + (size_t)nrhs * c->g.nif, c->pade_gt, c->st));
      g = c->pade_gt;
    }
    const double elems = (double)c->ndom * c->g.nloc * local_if_len(c->g);
    if (nrhs < kMatrixRhs) {
      // only the columns of faces that carry a trace are read: nloc entries per interface entry
      const double used = (double)c->g.nloc * c->g.nif;
      ProfScope ps(c, HBJ_K_LIFT, nrhs * used * 16.0, nrhs * used * 8.0);
      HIPCHK(launch_recon_dense(c->g, c->ft, c->coef, c->Wl, g, c->nzf, nrhs, u, c->st));
      return HBJ_OK;
    }
    // many right-hand sides: W_s is read once per subdomain for all of them (MFMA products)
    const int rpad = (nrhs + 15) / 16 * 16;
    const size_t need = (size_t)c->ndom * local_if_len(c->g) * rpad;
    if (need > c->Gbuf_cap) {
      dfree(c->Gbuf);
      c->Gbuf = nullptr;
      c->Gbuf_cap = 0;
      if (dalloc(&c->Gbuf, need)) return fail(HBJ_ENOMEM, "reconstruction workspace allocation failed");
      c->Gbuf_cap = need;
    }
    ProfScope ps(c, HBJ_K_LIFT, elems * 16.0, nrhs * elems * 8.0);
    HIPCHK(launch_recon_mm(c->g, c->coef, c->ft, c->Wl, g, c->nzf, nrhs, c->Gbuf, u, c->st));
    return HBJ_OK;
  }
  SolveIO io{};
  io.f = f;
  io.g_a = (c->g.nif > 0) ? g : nullptr;
  io.u = u;
  return run_solves<double>(c, S->dev + S->all_first, S->all_count, io, S->tiles + S->all_tile_first, S->all_tile_count);
}

int check_ready(hbj_ctx* c) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (!c->factored) return fail(HBJ_ESTATE, "hbj_factor has not run (or the medium changed)");
  return HBJ_OK;
}

// out = (I - S) g, FP64 local solves
// sub (only where op_sub_ok): out = (I - S) g - sub
int op_fp64(hbj_ctx* c, Schedule* S, const double2* g, double2* out, const double2* sub = nullptr) {
  SolveIO io{};
  io.g_a = g;
  io.tr_dst = out;
  io.tr_base = g;
  io.tr_sign = -1.0;
  io.tr_reflect = 1;
  io.tr_sub = sub;
  if (c->dense && df_enabled(c, S)) {
    DfArgs A{};
    A.st[2] = df_stage(g, g, out, g, -1.0, 0xF, 0);
    return run_df<double2>(c, S, DF_OP, A, c->T64);
  }
  if (c->dense)
    return run_dense(c, S->dev + S->all_first, S->eft + S->all_first, S->all_count, 0xF, io, false, S->all_dense_elems,
                     S->subs + S->all_sub_first, S->all_sub_count, S->nrhs, 0);
  return run_solves<double>(c, S->dev + S->all_first, S->all_count, io, S->tiles + S->all_tile_first, S->all_tile_count);
}

// sweeps over the precomputed steps; in = pass input, out = pass output (pre-filled with in)
// A pass whose output needs no pre-filling: dense operators on few right-hand sides write
// out = in + contribution and pass the other incoming positions through (copy mode).
bool pass_copies(const hbj_ctx* c, const Schedule* S) { return c->dense && S->nrhs < kMatrixRhs; }

// the operator rows of backward-pass chunk k into w = out - S out (out: the pass output)
int op_chunk(hbj_ctx* c, const Schedule* S, int k, const double2* z, double2* w) {
  SolveIO io{};
  io.g_a = z;
  io.tr_dst = w;
  io.tr_base = z;
  io.tr_sign = -1.0;
  io.tr_reflect = 1;
  return run_dense(c, S->dev + S->ov_first[k], S->eft + S->ov_first[k], S->ov_count[k], 0xF, io, false, 0.0);
}

// with opw (backward pass of a planned overlap): after step k the operator rows that the pass has
// finalised run on the operator stream, behind an event of the step; the last chunk runs on the
// context stream after the pass, which then waits for the operator stream
template <typename R>
int run_pass(hbj_ctx* c, const Schedule* S, const std::vector<Step>& steps, const double2* in, double2* out,
             int mask, double2* opw = nullptr, int chain_pass = -1) {
  Entry* dev = S->dev;
  const bool cp = pass_copies(c, S);
  const int nk = (int)steps.size();
  typedef typename Cplx<R>::T C;
  const Schedule::Chain* ch = chain_pass >= 0 ? &S->chain[chain_pass] : nullptr;
  if (ch) {  // the gathered tiles of every step, for the positions the previous step does not write
    const int rpad = (S->nrhs + 15) / 16 * 16;
    HIPCHK(launch_pregather<C>(ch->jdst, ch->jpos, ch->njobs, in, c->g.nif, S->nrhs, rpad, (C*)c->chain_buf, c->st));
  }
  if (opw) {
    if (!c->opst) HIPCHK(hipStreamCreateWithFlags(&c->opst, hipStreamNonBlocking));
    while ((int)c->ov_ev.size() < nk + 1) {
      hipEvent_t e = nullptr;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c->ov_ev.push_back(e);
    }
  }
  for (size_t si = 0; si < steps.size(); ++si) {
    const Step& s = steps[si];
    SolveIO io{};
    io.g_a = in;
    io.g_b = out;
    io.tr_dst = out;
    io.tr_base = cp ? in : out;
    io.in_faces = cp ? mask : 0;
    io.copy = cp ? 1 : 0;
    io.tr_sign = 1.0;
    io.tr_reflect = 1;
    const void* Gpre = nullptr;
    if (ch) {
      C* tiles = (C*)c->chain_buf;
      Gpre = tiles + ch->tile_off[si];
      if ((int)si + 1 < nk) {
        io.cmap = ch->cmap + si * (size_t)c->g.nif;
        io.ctile = tiles + ch->tile_off[si + 1];
        io.crpad = (S->nrhs + 15) / 16 * 16;
      }
    }
    int rc = c->dense ? run_dense(c, dev + s.first, S->eft + s.first, s.count, mask, io, sizeof(R) == 4, s.dense_elems,
                                  S->subs + s.sub_first, s.sub_count, S->nrhs, si == 0 ? 0 : 1,
                                  s.sarg >= 0 ? &S->sargs[s.sarg] : nullptr, Gpre)
                      : run_solves<R>(c, dev + s.first, s.count, io, S->tiles + s.tile_first, s.tile_count);
    if (rc) return rc;
    if (opw && (int)si + 1 < nk && S->ov_count[si] > 0) {
      HIPCHK(hipEventRecord(c->ov_ev[si], c->st));
      HIPCHK(hipStreamWaitEvent(c->opst, c->ov_ev[si], 0));
      hipStream_t keep = c->st;
      c->st = c->opst;
      rc = op_chunk(c, S, (int)si, out, opw);
      c->st = keep;
      if (rc) return rc;
    }
  }
  if (opw) {
    if (S->ov_count[nk - 1] > 0) {
      int rc = op_chunk(c, S, nk - 1, out, opw);
      if (rc) return rc;
    }
    HIPCHK(hipEventRecord(c->ov_ev[nk], c->opst));
    HIPCHK(hipStreamWaitEvent(c->st, c->ov_ev[nk], 0));
  }
  return HBJ_OK;
}

int op_apply(hbj_ctx* c, Schedule* S, const double2* g, double2* out, const double2* sub = nullptr);

// w: also apply the operator, w = (I - S) z, overlapped with the backward pass (the schedule
// planned it; the caller checked op_overlap_ok)
// Chained sweep steps (Schedule::Chain) for pass 0 (forward) or 1 (backward).  A position that step t
// reads is written by step t - 1 (its output then goes straight into step t's tile) or by no step
// up to t (the value at the pass start holds: it is gathered then); a schedule where some position
// read by step t was written by an earlier step, or twice, stays unchained.  Needs the passes in
// place (the pass input is the output) and the many-right-hand-side steps.
int build_chain(hbj_ctx* c, Schedule* S, int pass) {
  Schedule::Chain& ch = S->chain[pass];
  if (ch.built) return HBJ_OK;
  ch.built = true;
  const std::vector<Step>& steps = pass == 0 ? S->fwd : S->bwd;
  const int mask = pass == 0 ? kMaskFwd : kMaskBwd;
  const Geom& g = c->g;
  const int nk = (int)steps.size(), nif = g.nif, L = local_if_len(g);
  const int rpad = (S->nrhs + 15) / 16 * 16;
  if (nk == 0) return HBJ_OK;
  std::vector<int> wstep(nif, -1);  // the step of the pass writing each position
  for (int t = 0; t < nk; ++t) {
    const Step& st = steps[t];
    for (int q = 0; q < st.sub_count; ++q) {
      const FaceTab& F = c->ft_host[S->subs_host[st.sub_first + q]];
      for (int f = 0; f < 4; ++f) {
        if (!((mask >> f) & 1) || F.out_off[f] < 0) continue;
        for (int e = 0; e < face_len(g, f); ++e) {
          int& w = wstep[F.out_off[f] + e];
          if (w >= 0) return HBJ_OK;
          w = t;
        }
      }
    }
  }
  std::vector<size_t> off(nk + 1, 0);
  for (int t = 0; t < nk; ++t) off[t + 1] = off[t] + (size_t)steps[t].sub_count * L * rpad;
  std::vector<int32_t> cmap((size_t)nk * nif, -1);
  std::vector<int64_t> jdst;
  std::vector<int32_t> jpos;
  for (int t = 0; t < nk; ++t) {
    const Step& st = steps[t];
    for (int j = 0; j < st.sub_count; ++j) {
      const FaceTab& F = c->ft_host[S->subs_host[st.sub_first + j]];
      for (int f = 0; f < 4; ++f) {
        if (F.in_off[f] < 0) continue;
        for (int e = 0; e < face_len(g, f); ++e) {
          const int p = F.in_off[f] + e, w = wstep[p];
          const int slot = j * L + face_off(g, f) + e;
          if (t > 0 && w == t - 1) {
            cmap[(size_t)(t - 1) * nif + p] = slot;
          } else if (w < 0 || w > t) {
            jdst.push_back((int64_t)off[t] + (int64_t)slot * rpad);
            jpos.push_back(p);
          } else {
            return HBJ_OK;
          }
        }
      }
    }
  }
  HIPCHK(dalloc(&ch.cmap, cmap.size()));
  HIPCHK(hipMemcpyAsync(ch.cmap, cmap.data(), cmap.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  ch.njobs = (int)jpos.size();
  if (ch.njobs > 0) {
    HIPCHK(dalloc(&ch.jdst, jdst.size()));
    HIPCHK(dalloc(&ch.jpos, jpos.size()));
    HIPCHK(hipMemcpyAsync(ch.jdst, jdst.data(), jdst.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(ch.jpos, jpos.data(), jpos.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  }
  HIPCHK(hipStreamSynchronize(c->st));  // the host tables go out of scope
  ch.tile_off = off;
  ch.ok = true;
  return HBJ_OK;
}

template <typename R>
int precond_impl(hbj_ctx* c, Schedule* S, const double2* r, double2* z, int nrhs, double2* w = nullptr) {
  const size_t n = (size_t)nrhs * c->g.nif;
  int rc = ensure_pc(c, nrhs);
  if (rc) return rc;
  double2* y = c->pc_y;
  if (df_enabled(c, S)) {
    typedef typename Cplx<R>::T C;
    const C* T;
    if constexpr (sizeof(R) == 8) T = c->T64;
    else T = c->T32;
    const bool additive = c->P.bj_combine == HBJ_BJ_ADDITIVE;
    const bool residual = c->P.bj_compose == HBJ_BJ_RESIDUAL && c->fblocks.size() > 1;
    DfArgs A{};
    A.st[0] = df_stage(r, y, y, r, 1.0, kMaskFwd, 1);
    if (!additive && !residual) {
      A.st[1] = df_stage(y, z, z, y, 1.0, kMaskBwd, 1);
      return run_df<C>(c, S, DF_PC, A, T);
    }
    rc = run_df<C>(c, S, DF_FWD, A, T);
    if (rc) return rc;
    if (additive) HIPCHK(launch_add_ranges(y, r, c->ranges_f, c->nranges_f, c->g.nif, nrhs, c->st));
    const double2* bin = y;
    if (residual) {
      double2* t = c->pc_t;
      rc = op_apply(c, S, y, t);
      if (rc) return rc;
      HIPCHK(launch_axpby(t, r, mk(1.0, 0.0), mk(-1.0, 0.0), n, c->st));  // t = r - (I - S) y
      bin = t;
    }
    A.st[1] = df_stage(bin, z, z, bin, 1.0, kMaskBwd, 1);
    rc = run_df<C>(c, S, DF_BWD, A, T);
    if (rc) return rc;
    if (additive) HIPCHK(launch_add_ranges(z, bin, c->ranges_b, c->nranges_b, c->g.nif, nrhs, c->st));
    if (residual) HIPCHK(launch_axpby(z, y, mk(1.0, 0.0), mk(1.0, 0.0), n, c->st));
    return HBJ_OK;
  }
  const bool cp = pass_copies(c, S);
  // Both passes in place on z pre-filled with r (dense operators, the default readings, no two
  // neighbouring subdomains in a step): a step writes each of its outgoing positions once, reading
  // the old value there as the base of that write, and reads incoming positions that no step of
  // the pass writes or that an earlier step wrote, as from a separate pass output pre-filled with
  // the pass input.  One copy of the vector less per application.
  if (!cp && c->dense && S->steps_apart && !w && c->P.bj_combine == HBJ_BJ_RESTRICTED &&
      !(c->P.bj_compose == HBJ_BJ_RESIDUAL && c->fblocks.size() > 1)) {
    HIPCHK(launch_copy(z, r, n, c->st));
    // many right-hand sides with tiles of gathered incoming data (or no variant chosen yet): the
    // steps pass their outputs on to the next step's tile instead of a gather launch per step
    bool chain = false;
    if (S->nrhs >= kMatrixRhs && c->chain_ok) {
      const int v = c->mm_variant[sizeof(R) == 4 ? 2 : 0];
      if (v < 0 || mm_variant_gathered(v)) {
        rc = build_chain(c, S, 0);
        if (!rc) rc = build_chain(c, S, 1);
        if (rc) return rc;
        chain = S->chain[0].ok && S->chain[1].ok;
        if (chain) {
          typedef typename Cplx<R>::T C;
          const size_t need = std::max(S->chain[0].tile_off.back(), S->chain[1].tile_off.back()) * sizeof(C);
          if (need > c->chain_cap) {
            dfree(c->chain_buf);
            c->chain_buf = nullptr;
            c->chain_cap = 0;
            if (hipMalloc(&c->chain_buf, need) != hipSuccess) return fail(HBJ_ENOMEM, "tile buffer allocation failed");
            c->chain_cap = need;
          }
        }
      }
    }
    rc = run_pass<R>(c, S, S->fwd, z, z, kMaskFwd, nullptr, chain ? 0 : -1);
    if (rc) return rc;
    return run_pass<R>(c, S, S->bwd, z, z, kMaskBwd, nullptr, chain ? 1 : -1);
  }
  if (!cp) HIPCHK(launch_copy(y, r, n, c->st));
  rc = run_pass<R>(c, S, S->fwd, r, y, kMaskFwd);
  if (rc) return rc;
  if (c->P.bj_combine == HBJ_BJ_ADDITIVE) HIPCHK(launch_add_ranges(y, r, c->ranges_f, c->nranges_f, c->g.nif, nrhs, c->st));
  if (c->P.bj_compose == HBJ_BJ_RESIDUAL && c->fblocks.size() > 1) {
    // r_half = r - (I - S) y ; z = y + B_U^{-1} r_half
    double2* t = c->pc_t;
    rc = op_apply(c, S, y, t);
    if (rc) return rc;
    HIPCHK(launch_axpby(t, r, mk(1.0, 0.0), mk(-1.0, 0.0), n, c->st));  // t = r - t
    if (!cp) HIPCHK(launch_copy(z, t, n, c->st));
    rc = run_pass<R>(c, S, S->bwd, t, z, kMaskBwd);
    if (rc) return rc;
    if (c->P.bj_combine == HBJ_BJ_ADDITIVE)
      HIPCHK(launch_add_ranges(z, t, c->ranges_b, c->nranges_b, c->g.nif, nrhs, c->st));
    HIPCHK(launch_axpby(z, y, mk(1.0, 0.0), mk(1.0, 0.0), n, c->st));
    return HBJ_OK;
  }
  if (!cp) HIPCHK(launch_copy(z, y, n, c->st));
  rc = run_pass<R>(c, S, S->bwd, y, z, kMaskBwd, w);
  if (rc) return rc;
  if (c->P.bj_combine == HBJ_BJ_ADDITIVE) HIPCHK(launch_add_ranges(z, y, c->ranges_b, c->nranges_b, c->g.nif, nrhs, c->st));
  return HBJ_OK;
}

int precond(hbj_ctx* c, Schedule* S, const double2* r, double2* z, int nrhs) {
  const size_t n = (size_t)nrhs * c->g.nif;
  if (c->P.precond == HBJ_PC_NONE || c->ndom == 1) {
    HIPCHK(launch_copy(z, r, n, c->st));
    return HBJ_OK;
  }
  if (c->P.precision == HBJ_MIXED) return precond_impl<float>(c, S, r, z, nrhs);
  return precond_impl<double>(c, S, r, z, nrhs);
}

}  // namespace

// mixed-precision operator: local solves with complex64 factors refined to FP64 accuracy
int op_mixed(hbj_ctx* c, Schedule* S, const double2* g, double2* out);

namespace {
int op_apply(hbj_ctx* c, Schedule* S, const double2* g, double2* out, const double2* sub) {
  if (sub) return op_fp64(c, S, g, out, sub);  // dense operators (op_sub_ok): complex128 in both precisions
  if (c->P.precision == HBJ_MIXED) return op_mixed(c, S, g, out);
  return op_fp64(c, S, g, out);
}

// Whether the operator can subtract a vector in its own epilogue: the dense operators applied on
// the matrix-product path (many right-hand sides, stepped sweeps)
bool op_sub_ok(const hbj_ctx* c, const Schedule* S) {
  return c->dense && !df_enabled(c, S) && S->nrhs >= kMatrixRhs;
}

// The operator rows run beside the backward pass when the schedule planned it (dense operators,
// few right-hand sides, stepped sweeps, default readings) and no launch is profiled or captured.
bool op_overlap_ok(const hbj_ctx* c, const Schedule* S) {
  return c->op_overlap && S->ov_ok && c->dense && !c->prof && !c->use_graphs && !df_enabled(c, S) &&
         c->P.precond != HBJ_PC_NONE && c->ndom > 1 && S->nrhs < kMatrixRhs;
}

// z = P^{-1} v, w = (I - S) z: one dataflow launch for the FP64 dense form with the default
// readings, the two calls otherwise (the operator overlapped with the backward pass where it can)
int pc_op(hbj_ctx* c, Schedule* S, const double2* v, double2* z, double2* w, int nrhs, const double2* sub = nullptr) {
  const bool fused = df_enabled(c, S) && c->P.precision == HBJ_FP64 && c->P.precond != HBJ_PC_NONE &&
                     c->ndom > 1 && c->P.bj_combine == HBJ_BJ_RESTRICTED &&
                     !(c->P.bj_compose == HBJ_BJ_RESIDUAL && c->fblocks.size() > 1);
  if (!fused) {
    if (op_overlap_ok(c, S)) {
      if (c->P.precision == HBJ_MIXED) return precond_impl<float>(c, S, v, z, nrhs, w);
      return precond_impl<double>(c, S, v, z, nrhs, w);
    }
    int rc = precond(c, S, v, z, nrhs);
    if (rc) return rc;
    return op_apply(c, S, z, w, sub);
  }
  int rc = ensure_pc(c, nrhs);
  if (rc) return rc;
  double2* y = c->pc_y;
  DfArgs A{};
  A.st[0] = df_stage(v, y, y, v, 1.0, kMaskFwd, 1);
  A.st[1] = df_stage(y, z, z, y, 1.0, kMaskBwd, 1);
  A.st[2] = df_stage(z, z, w, z, -1.0, 0xF, 0);
  return run_df<double2>(c, S, DF_PC_OP, A, c->T64);
}
}  // namespace

// ===========================================================================
// mixed precision: iterative refinement of the operator's local solves
// ===========================================================================
hipError_t launch_build_rhs(const Geom& g, const Entry* ent, int nent, const FaceTab* ft, const IfCoef* coef,
                            const SolveIO& io, double2* rhs64, hipStream_t st);
hipError_t launch_axpy_c64(double2* x64, const float2* dx, const Geom& g, const SolveLayout& L, int nent,
                           hipStream_t st);

// Refinement of the operator's complex64 local solves: at most kLocalSolvesMax solves per local
// problem; a step counts as progress when the largest relative local residual ||r|| / ||rhs||
// falls below half of the previous one, and refinement stops once it is below kLocalResidTarget
// (FP64 level) or stops making progress (its floor, about eps64 cond(A_s), is then reached).
static const int kLocalSolvesMax = 8;
static const double kLocalResidTarget = 1e-14;

int op_mixed(hbj_ctx* c, Schedule* S, const double2* g, double2* out) {
  if (c->dense) return op_fp64(c, S, g, out);  // the complex128 dense operator is exact already
  const Entry* ent = S->dev + S->all_first;
  const int nent = S->all_count;
  int rc = ensure_loc64(c, nent);
  if (rc) return rc;
  rc = ensure_ybuf(c, nent, sizeof(float2));
  if (rc) return rc;
  if ((size_t)nent > c->ir_ratio_cap) {
    dfree(c->ir_ratio);
    c->ir_ratio = nullptr;
    c->ir_ratio_cap = 0;
    if (dalloc(&c->ir_ratio, (size_t)nent)) return fail(HBJ_ENOMEM, "refinement workspace allocation failed");
    c->ir_ratio_cap = nent;
  }
  SolveIO io{};
  io.g_a = g;
  HIPCHK(launch_build_rhs(c->g, ent, nent, c->ft, c->coef, io, c->rhs64, c->st));
  HIPCHK(launch_fill_zero(c->x64, (size_t)nent * c->g.nloc * sizeof(double2), c->st));
  HIPCHK(launch_copy(c->r64, c->rhs64, (size_t)nent * c->g.nloc, c->st));
  std::vector<double> ratio(nent);
  double prev = 1.0;
  int nsolves = 0;
  for (int it = 0; it < kLocalSolvesMax; ++it) {
    SolveIO lio{};
    lio.rhs64 = c->r64;
    rc = launch_solve_pair<float>(c, ent, nent, S->tiles + S->all_tile_first, S->all_tile_count, lio, c->mf32,
                                  c->mb32);
    if (rc) return rc;
    c->local_solves += nent;
    ++nsolves;
    HIPCHK(launch_axpy_c64(c->x64, (const float2*)c->ybuf, c->g, c->L, nent, c->st));
    HIPCHK(launch_local_residual(c->g, ent, nent, c->ft, c->band, c->diag, c->rhs64, c->x64, c->r64, c->st));
    HIPCHK(launch_entry_ratio(c->r64, c->rhs64, c->g.nloc, nent, c->ir_ratio, c->st));
    HIPCHK(hipMemcpyAsync(ratio.data(), c->ir_ratio, nent * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const double worst = *std::max_element(ratio.begin(), ratio.end());
    c->last_ir_resid = worst;
    if (worst <= kLocalResidTarget || worst > 0.5 * prev) break;
    prev = worst;
  }
  c->last_ir = nsolves;
  c->ir_max = std::max(c->ir_max, nsolves);
  c->ir_resid_max = std::max(c->ir_resid_max, c->last_ir_resid);
  SolveIO tio{};
  tio.g_a = g;
  tio.tr_dst = out;
  tio.tr_base = g;
  tio.tr_sign = -1.0;
  tio.tr_reflect = 1;
  HIPCHK(launch_emit_traces(c->g, ent, nent, c->ft, c->band, tio, c->x64, c->st));
  return HBJ_OK;
}

// ===========================================================================
// GMRES / FGMRES, right preconditioned, columns in lockstep
// ===========================================================================
namespace {

struct Gmres {
  hbj_ctx* c;
  Schedule* S;
  int ncol, nif, m;
  bool flexible;
  // device
  double2 *V = nullptr, *Z = nullptr, *w = nullptr, *b = nullptr, *x = nullptr, *r = nullptr, *zt = nullptr;
  double2 *hbuf = nullptr, *h1 = nullptr, *h2 = nullptr, *ydev = nullptr, *partial = nullptr;
  double *nrm = nullptr, *npartial = nullptr;
  size_t hbuf_len = 0;
  int nchunk = 0;   // chunks of the inner-product pass (classical Gram-Schmidt twice)
  int nchunk2 = 0;  // the same for the delayed-reorthogonalisation pass (twice as many products)
  std::vector<hipGraphExec_t> graphs;  // iteration j of a restart cycle, captured at first use
  int graph_epoch = -1;
  // s-step cycles: inner-product partials, the coefficient records and their pinned host copy
  double2 *bpart = nullptr, *coef = nullptr, *coef_host = nullptr;
  size_t bpart_elems = 0;
  double2* hbuf_host = nullptr;        // pinned host h1 | h2 | norms, two slots (step j uses slot j & 1)
  double2* hbuf_mapped = nullptr;      // the same memory as the kernels address it
  hipEvent_t ev_h[2] = {nullptr, nullptr};
  double2* slot(int j) { return hbuf_host + (size_t)(j & 1) * hbuf_len; }
  double2* slot_dev(int j) { return hbuf_mapped + (size_t)(j & 1) * hbuf_len; }
  void drop_graphs() {
    for (auto& ge : graphs)
      if (ge) (void)hipGraphExecDestroy(ge);
    graphs.assign(graphs.size(), nullptr);
  }
  bool matches(const Schedule* S_, int ncol_, int nif_, int m_, bool flexible_) const {
    return S == S_ && ncol == ncol_ && nif == nif_ && m == m_ && flexible == flexible_;
  }
  ~Gmres() {
    drop_graphs();
    for (auto& e : ev_h)
      if (e) (void)hipEventDestroy(e);
    if (hbuf_host) (void)hipHostFree(hbuf_host);
    if (coef_host) (void)hipHostFree(coef_host);
    for (void* p : {(void*)V, (void*)Z, (void*)w, (void*)b, (void*)x, (void*)r, (void*)zt, (void*)hbuf,
                    (void*)ydev, (void*)partial, (void*)npartial, (void*)bpart, (void*)coef})
      dfree(p);
  }
  int alloc_sstep() {
    if (coef) return HBJ_OK;
    bpart_elems = bgs_partial_elems(nif, ncol);
    if (dalloc(&bpart, bpart_elems) || dalloc(&coef, (size_t)ncol * kSstepCoefLd))
      return fail(HBJ_ENOMEM, "s-step workspace allocation failed");
    if (hipHostMalloc((void**)&coef_host, (size_t)ncol * kSstepCoefLd * sizeof(double2), 0) != hipSuccess)
      return fail(HBJ_ENOMEM, "s-step host buffer allocation failed");
    return HBJ_OK;
  }
  size_t vs() const { return (size_t)ncol * nif; }
  double2* Vi(int i) { return V + (size_t)i * vs(); }
  double2* Zi(int i) { return Z + (size_t)i * vs(); }

  int alloc() {
    // every chunk fits one workgroup's registers in the fused dot kernel (256 threads x 4)
    // chunks of about 1024 entries, few enough that the fused update holds all partials
    nchunk = std::max(1, std::min((nif + 1023) / 1024, 2048 / (m + 1)));
    nchunk2 = std::max(1, std::min((nif + 1023) / 1024, 2048 / (2 * m + 3)));
    // h1 | h2 | norms (classical Gram-Schmidt twice) or a | c | (nu, s, |w|^2, 0) per column
    hbuf_len = 2 * (size_t)ncol * (m + 1) + 2 * (size_t)ncol;
    const size_t npart = std::max((size_t)(m + 1) * nchunk, (size_t)(2 * m + 3) * nchunk2);
    const size_t nblk = ((size_t)nif + 255) / 256;
    if (dalloc(&V, (size_t)(m + 1) * vs()) || (flexible && dalloc(&Z, (size_t)m * vs())) || dalloc(&w, vs()) ||
        dalloc(&b, vs()) || dalloc(&x, vs()) || dalloc(&r, vs()) || dalloc(&zt, vs()) || dalloc(&hbuf, hbuf_len) ||
        dalloc(&ydev, (size_t)ncol * (m + 1)) || dalloc(&partial, (size_t)ncol * npart) ||
        dalloc(&npartial, (size_t)ncol * std::max<size_t>(nchunk, nblk)))
      return fail(HBJ_ENOMEM, "GMRES workspace allocation failed");
    // coherent pinned memory: the Gram-Schmidt kernels store h and the norms straight into it, and
    // the stores are visible to the host once the step's completion event has fired
    if (hipHostMalloc((void**)&hbuf_host, 2 * hbuf_len * sizeof(double2), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
      return fail(HBJ_ENOMEM, "GMRES host buffer allocation failed");
    if (hipHostGetDevicePointer((void**)&hbuf_mapped, hbuf_host, 0) != hipSuccess)
      return fail(HBJ_EHIP, "GMRES host buffer mapping failed");
    for (auto& e : ev_h)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return fail(HBJ_EHIP, "event creation failed");
    graphs.assign(m, nullptr);
    // h1 | h2 | norms in one buffer: one copy to the host per iteration
    h1 = hbuf;
    h2 = hbuf + (size_t)ncol * (m + 1);
    nrm = (double*)(hbuf + 2 * (size_t)ncol * (m + 1));
    return HBJ_OK;
  }

  int norms(const double2* v, std::vector<double>& out) {
    HIPCHK(launch_norms(v, nif, ncol, npartial, nchunk, c->st));
    HIPCHK(launch_reduce_norms(npartial, ncol, nchunk, nrm, c->st));
    out.resize(ncol);
    HIPCHK(hipMemcpyAsync(out.data(), nrm, ncol * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return HBJ_OK;
  }
};

void destroy_gmres(Gmres* g) { delete g; }

// Whether step j stores h1 | h2 | norms straight into its pinned host slot (the fused kernels
// publish them themselves) or into G.hbuf, from where the caller copies them.
bool h_direct(const Gmres& G, int j) { return krylov_fusable(j + 1, G.nchunk, G.nif); }

// One Arnoldi step for column block j: z = P^{-1} V_j, w = (I - S) z, classical Gram-Schmidt with
// one reorthogonalisation, V_{j+1} = w / ||w||; h1, h2 and the norm land in host slot j & 1
// (h_direct) or in G.hbuf.
int arnoldi_kernels(hbj_ctx* c, Schedule* S, Gmres& G, int j) {
  const int ncol = G.ncol, nif = G.nif, m = G.m;
  const size_t vs = G.vs();
  double2* z = G.flexible ? G.Zi(j) : G.zt;
  int rc = pc_op(c, S, G.Vi(j), z, G.w, ncol);
  if (rc) return rc;
  ProfScope ps(c, HBJ_K_KRYLOV, 4.0 * (j + 1) * vs * 16.0 + 2.0 * vs * 16.0, 16.0 * (j + 1) * vs);
  if (h_direct(G, j)) {
    // 5 launches: dots, update (+ h1), dots, update (+ h2, |w|^2 partials), norm + scaling
    double2* hs = G.slot_dev(j);
    double2* h1 = hs;
    double2* h2 = hs + (size_t)ncol * (m + 1);
    double* nrm = (double*)(hs + 2 * (size_t)ncol * (m + 1));
    HIPCHK(launch_multidot(G.V, vs, j + 1, G.w, nif, ncol, G.partial, G.nchunk, c->st));
    HIPCHK(launch_update_reduce(G.w, G.V, vs, j + 1, G.partial, G.nchunk, h1, m + 1, mk(-1.0, 0.0), nif, ncol,
                                nullptr, c->st));
    HIPCHK(launch_multidot(G.V, vs, j + 1, G.w, nif, ncol, G.partial, G.nchunk, c->st));
    HIPCHK(launch_update_reduce(G.w, G.V, vs, j + 1, G.partial, G.nchunk, h2, m + 1, mk(-1.0, 0.0), nif, ncol,
                                G.npartial, c->st));
    HIPCHK(launch_scale_reduce(G.Vi(j + 1), G.w, G.npartial, nrm, nif, ncol, c->st));
  } else {
    HIPCHK(launch_multidot(G.V, vs, j + 1, G.w, nif, ncol, G.partial, G.nchunk, c->st));
    HIPCHK(launch_reduce_partials(G.partial, j + 1, ncol, G.nchunk, G.h1, m + 1, mk(1.0, 0.0), c->st));
    HIPCHK(launch_update(G.w, G.V, vs, j + 1, G.h1, m + 1, mk(-1.0, 0.0), nif, ncol, c->st));
    HIPCHK(launch_multidot(G.V, vs, j + 1, G.w, nif, ncol, G.partial, G.nchunk, c->st));
    HIPCHK(launch_reduce_partials(G.partial, j + 1, ncol, G.nchunk, G.h2, m + 1, mk(1.0, 0.0), c->st));
    HIPCHK(launch_update(G.w, G.V, vs, j + 1, G.h2, m + 1, mk(-1.0, 0.0), nif, ncol, c->st));
    HIPCHK(launch_norms(G.w, nif, ncol, G.npartial, G.nchunk, c->st));
    HIPCHK(launch_reduce_norms(G.npartial, ncol, G.nchunk, G.nrm, c->st));
    HIPCHK(launch_scale_by_inv(G.Vi(j + 1), G.w, G.nrm, nif, ncol, c->st));
  }
  return HBJ_OK;
}

// Delayed reorthogonalisation when asked for and when the restart length fits its fused kernels;
// the choice holds for a whole solve.
// s-step cycles when asked for, with flexible storage (the solution is formed from the kept
// preconditioned vectors) and a basis that fits the block kernels; delayed reorthogonalisation
// otherwise
// (HBJ_ORTH_AUTO: for column blocks of at least 2^20 entries, where a pass over the basis outweighs
// the per-block costs: the shift launch per step, the host round trip per block, the unused steps
// of the last block; measured on MI355X: 64 right-hand sides at 2048^2 gain 25%, 16 at 512^2 and
// one at 1024^2 lose)
constexpr size_t kSstepAutoElems = size_t(1) << 20;
bool use_sstep(const hbj_ctx* c, const Gmres& G) {
  const bool want = c->orth == HBJ_ORTH_SSTEP || (c->orth == HBJ_ORTH_AUTO && G.vs() >= kSstepAutoElems);
  return want && G.flexible && G.m + 1 <= kSstepMaxBasis;
}
bool use_dcgs(const hbj_ctx* c, const Gmres& G) {
  return c->orth != HBJ_ORTH_CGS2 && !use_sstep(c, G) && dcgs_fits(G.m, G.nchunk2);
}

// Arnoldi step j with delayed reorthogonalisation: z = P^{-1} x_j (x_j = V_j after one
// Gram-Schmidt pass), w = (I - S) z, one inner-product pass and one update pass (v_j into V_j,
// x_{j+1} into V_{j+1}); the coefficients go to host slot j & 1.  finish: the step that closes a
// restart cycle, which only needs the coefficients of x_j (no preconditioner, operator or update).
int arnoldi_kernels_dcgs(hbj_ctx* c, Schedule* S, Gmres& G, int j, bool finish) {
  const int ncol = G.ncol, nif = G.nif, m = G.m;
  const size_t vs = G.vs();
  double2* x = G.Vi(j);
  if (!finish) {
    double2* z = G.flexible ? G.Zi(j) : G.zt;
    int rc = pc_op(c, S, x, z, G.w, ncol);
    if (rc) return rc;
  }
  // algorithmic bytes: the inner-product pass reads V_0..V_{j-1}, x and w; the update pass reads
  // them again and writes v_j and x_{j+1}
  ProfScope ps(c, HBJ_K_KRYLOV, (finish ? j + 1.0 : 2.0 * j + 6.0) * vs * 16.0, (finish ? 8.0 : 32.0) * j * vs);
  const double2* w = finish ? x : G.w;
  HIPCHK(launch_dots2(G.V, vs, j, x, w, nif, ncol, G.partial, G.nchunk2, c->st));
  HIPCHK(launch_dcgs_update(G.V, vs, j, x, finish ? nullptr : G.Vi(j + 1), w, G.partial, G.nchunk2, G.slot_dev(j),
                            m + 1, nif, ncol, finish, c->st));
  return HBJ_OK;
}

int step_kernels(hbj_ctx* c, Schedule* S, Gmres& G, int j) {
  return use_dcgs(c, G) ? arnoldi_kernels_dcgs(c, S, G, j, false) : arnoldi_kernels(c, S, G, j);
}

// Iterations that are pure kernel launches on fixed buffers (dense operators, stepped sweeps,
// few right-hand sides: no allocation, tuning or host synchronisation inside) are captured
// once per step index j and replayed as one graph launch.
bool graphable(const hbj_ctx* c, const Schedule* S) {
  return c->use_graphs && !c->prof && c->dense && c->P.sweep_exec == HBJ_SWEEP_STEPPED && S->nrhs < kMatrixRhs;
}

int arnoldi_step(hbj_ctx* c, Schedule* S, Gmres& G, int j) {
  if (!graphable(c, S)) return step_kernels(c, S, G, j);
  if (G.graph_epoch != c->graph_epoch) {
    G.drop_graphs();
    G.graph_epoch = c->graph_epoch;
  }
  if (!G.graphs[j]) {
    if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    // the capture stream starts after everything queued so far on the context stream
    HIPCHK(hipEventRecord(c->ev0, c->st));
    HIPCHK(hipStreamWaitEvent(c->cap, c->ev0, 0));
    hipStream_t keep = c->st;
    c->st = c->cap;
    hipError_t he = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    int rc = (he == hipSuccess) ? step_kernels(c, S, G, j) : HBJ_OK;
    hipGraph_t gr = nullptr;
    const hipError_t he2 = (he == hipSuccess) ? hipStreamEndCapture(c->cap, &gr) : he;
    c->st = keep;
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (he2 != hipSuccess) return fail(HBJ_EHIP, hipGetErrorString(he2));
    hipGraphExec_t ex = nullptr;
    he = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (he != hipSuccess) return fail(HBJ_EHIP, hipGetErrorString(he));
    G.graphs[j] = ex;
  }
  HIPCHK(hipGraphLaunch(G.graphs[j], c->st));
  return HBJ_OK;
}

void givens(zc a, zc b, double& cs, zc& sn) {
  if (std::abs(b) == 0.0) { cs = 1.0; sn = 0.0; return; }
  if (std::abs(a) == 0.0) { cs = 0.0; sn = std::conj(b) / std::abs(b); return; }
  const double rr = std::hypot(std::abs(a), std::abs(b));
  cs = std::abs(a) / rr;
  sn = (a / std::abs(a)) * std::conj(b) / rr;
}

}  // namespace

static int gmres_solve(hbj_ctx* c, Schedule* S, Gmres& G, const hbj_solve_opts& o, hbj_solve_stats* stats,
                       std::vector<int>& col_iters, std::vector<double>& col_relres, std::vector<char>& col_conv,
                       std::vector<double>& hist) {
  const int ncol = G.ncol, nif = G.nif, m = G.m;
  const size_t vs = G.vs();
  std::vector<double> bnorm, rnorm;
  int rc = G.norms(G.b, bnorm);
  if (rc) return rc;
  col_iters.assign(ncol, 0);
  col_relres.assign(ncol, 0.0);
  col_conv.assign(ncol, 0);
  for (int k = 0; k < ncol; ++k)
    if (bnorm[k] == 0.0) col_conv[k] = 1;
  HIPCHK(launch_fill_zero(G.x, vs * sizeof(double2), c->st));
  HIPCHK(launch_copy(G.r, G.b, vs, c->st));
  rnorm = bnorm;
  hist.assign(1, 1.0);
  int total = 0;
  std::vector<zc> H((size_t)ncol * (m + 1) * m), e1((size_t)ncol * (m + 1)), sn((size_t)ncol * m);
  std::vector<double> cs((size_t)ncol * m);
  std::vector<double2> hh1((size_t)ncol * (m + 1)), hh2((size_t)ncol * (m + 1));
  std::vector<double> hn(ncol);
  std::vector<int> jc(ncol);
  std::vector<double2> yh((size_t)ncol * (m + 1));
  auto Hc = [&](int k, int i, int j) -> zc& { return H[((size_t)k * (m + 1) + i) * m + j]; };
  const bool sst = use_sstep(c, G);
  const bool dcgs = use_dcgs(c, G);
  // delayed reorthogonalisation: R (x_j = V R e_j), and c^(j), s_j, |w_j|^2 of the last step
  std::vector<zc> R(dcgs ? (size_t)ncol * m * m : 0), cprev(dcgs ? (size_t)ncol * (m + 1) : 0);
  std::vector<double> sprev(ncol), wwprev(ncol);
  // s-step cycles: residual reduction per step of each column over its last block (none yet: empty)
  std::vector<double> ss_rate;
  auto Rc = [&](int k, int i, int j) -> zc& { return R[((size_t)k * m + i) * m + j]; };
  while (true) {
    bool any = false;
    for (int k = 0; k < ncol; ++k) any |= !col_conv[k];
    if (!any || total >= o.maxit) break;
    // V_0 = r / ||r|| (zero for finished columns)
    std::vector<double> inv(ncol);
    for (int k = 0; k < ncol; ++k) inv[k] = col_conv[k] ? 0.0 : rnorm[k];
    HIPCHK(hipMemcpyAsync(G.nrm, inv.data(), ncol * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(launch_scale_by_inv(G.Vi(0), G.r, G.nrm, nif, ncol, c->st));
    std::vector<char> active(ncol);
    for (int k = 0; k < ncol; ++k) {
      active[k] = !col_conv[k];
      jc[k] = 0;
      std::fill(&e1[(size_t)k * (m + 1)], &e1[(size_t)k * (m + 1)] + m + 1, zc(0.0));
      e1[(size_t)k * (m + 1)] = rnorm[k];
    }
    if (sst) {
      // s-step cycle in blocks of sb steps.  Per block: sb preconditioner and operator applications
      // build y_{i+1} = (I - S) z_{k+i} - y_i with z_{k+i} = P^{-1} y_i (kept in Z) from y_0 = V_k,
      // in the slots V_{k+1..k+sb}; one block Gram-Schmidt turns them into orthonormal vectors there
      // (y_{l+1} = V_{<=k} C e_l + V_{k+1..k+sb} R e_l), and the host forms Hessenberg columns
      // k..k+sb-1 from (I - S) z_{k+i} = y_i + y_{i+1}.  The GPU idles only while the host reads a
      // block back (one block is many launches long); convergence is found at the exact step, the
      // remaining steps of that block being unused.
      rc = G.alloc_sstep();
      if (rc) return rc;
      const int kmax = std::min(m, o.maxit - total);
      const int ld = kSstepCoefLd;
      for (int k = 0; k < kmax;) {
        // A block that would end past the step where every column is predicted to converge (at
        // each column's residual reduction per step over its last block, one step of margin) is
        // shortened: the steps after convergence would be unused.  The prediction changes only the
        // block lengths, not the steps' iterates.
        int want = c->sstep_block;
        if (!ss_rate.empty()) {
          int need = 0;
          for (int q = 0; q < ncol && need < want; ++q) {
            if (!active[q]) continue;
            const double est = std::abs(e1[(size_t)q * (m + 1) + k]) / bnorm[q], rq = ss_rate[q];
            if (!(rq > 0.0 && rq < 1.0) || !(est > o.tol)) { need = want; break; }
            const double nd = std::ceil(std::log(o.tol / est) / std::log(rq)) + 1.0;
            need = std::max(need, (int)std::min<double>(want, nd));
          }
          want = std::max(1, std::min(want, need));
        }
        const int sb = std::min(want, kmax - k);
        // the shift (- y_i) in the operator's epilogue where it can take it, else one more launch
        const bool fold = op_sub_ok(c, S);
        for (int i = 0; i < sb; ++i) {
          rc = pc_op(c, S, G.Vi(k + i), G.Zi(k + i), G.Vi(k + i + 1), ncol, fold ? G.Vi(k + i) : nullptr);
          if (rc) return rc;
          if (fold) continue;
          ProfScope ps(c, HBJ_K_KRYLOV, 3.0 * vs * 16.0, 8.0 * vs);
          HIPCHK(launch_axpby(G.Vi(k + i + 1), G.Vi(k + i), mk(-1.0, 0.0), mk(1.0, 0.0), vs, c->st));
        }
        {
          // the inner-product pass reads V_0..V_{k+sb}; the update pass reads them again and writes sb
          ProfScope ps(c, HBJ_K_KRYLOV, (2.0 * (k + 1) + 3.0 * sb) * vs * 16.0, 16.0 * (k + 1 + sb) * sb * vs);
          HIPCHK(launch_bgs(G.V, vs, k + 1, sb, nif, ncol, G.bpart, G.bpart_elems, G.coef, ld, c->st));
        }
        const size_t row = (size_t)(129 + (k + 1) * kSstepMax) * sizeof(double2);
        HIPCHK(hipMemcpy2DAsync(G.coef_host, ld * sizeof(double2), G.coef, ld * sizeof(double2), row, ncol,
                                hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        bool any_active = false;
        if (ss_rate.empty()) ss_rate.assign(ncol, 0.0);
        for (int q = 0; q < ncol; ++q) {
          if (!active[q]) continue;
          const double2* cf = G.coef_host + (size_t)q * ld;
          // coefficient of basis vector r in y_i (y_0 = V_k)
          auto ycoef = [&](int i, int r) -> zc {
            if (i == 0) return r == k ? zc(1.0, 0.0) : zc(0.0, 0.0);
            const int l = i - 1;
            double2 v = mk(0.0, 0.0);
            if (r <= k) v = cf[129 + r * kSstepMax + l];
            else if (r - k - 1 <= l) v = cf[(r - k - 1) * kSstepMax + l];
            return zc(v.x, v.y);
          };
          double* csk = &cs[(size_t)q * m];
          zc* snk = &sn[(size_t)q * m];
          zc* ek = &e1[(size_t)q * (m + 1)];
          const double est0 = std::abs(ek[k]);
          int done = 0;
          for (int i = 0; i < sb && active[q]; ++i, ++done) {
            const int j = k + i;
            for (int r = 0; r <= j + 1; ++r) Hc(q, r, j) = ycoef(i, r) + ycoef(i + 1, r);
            const double hn = std::abs(Hc(q, j + 1, j));
            for (int r = 0; r < j; ++r) {
              const zc t = csk[r] * Hc(q, r, j) + snk[r] * Hc(q, r + 1, j);
              Hc(q, r + 1, j) = -std::conj(snk[r]) * Hc(q, r, j) + csk[r] * Hc(q, r + 1, j);
              Hc(q, r, j) = t;
            }
            givens(Hc(q, j, j), Hc(q, j + 1, j), csk[j], snk[j]);
            Hc(q, j, j) = csk[j] * Hc(q, j, j) + snk[j] * Hc(q, j + 1, j);
            Hc(q, j + 1, j) = 0.0;
            ek[j + 1] = -std::conj(snk[j]) * ek[j];
            ek[j] = csk[j] * ek[j];
            jc[q] = j + 1;
            col_iters[q] += 1;
            const double est = std::abs(ek[j + 1]) / bnorm[q];
            if (q == 0) hist.push_back(est);
            if (est <= o.tol || hn == 0.0 || std::abs(Hc(q, j, j)) == 0.0) active[q] = 0;
          }
          if (done > 0 && est0 > 0.0) ss_rate[q] = std::pow(std::abs(ek[k + done]) / est0, 1.0 / done);
          any_active |= active[q];
        }
        total += sb;
        k += sb;
        if (!any_active) break;
      }
    } else if (!dcgs) {
      // Step j + 1 is queued before the host reads step j back: it needs only V_{j+1}, already on
      // the device, so the GPU never waits for the host's Givens rotations. When the host finds
      // that every column has converged at step j, the queued step's results are simply unused.
      auto launch_step = [&](int jj) -> int {
        int r2 = arnoldi_step(c, S, G, jj);
        if (r2) return r2;
        if (!h_direct(G, jj))
          HIPCHK(hipMemcpyAsync(G.slot(jj), G.hbuf, G.hbuf_len * sizeof(double2), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipEventRecord(G.ev_h[jj & 1], c->st));
        return HBJ_OK;
      };
      int j = 0;
      if (m > 0 && total < o.maxit) {
        rc = launch_step(0);
        if (rc) return rc;
      }
      for (; j < m && total < o.maxit; ++j) {
        if (j + 1 < m && total + 1 < o.maxit) {
          rc = launch_step(j + 1);
          if (rc) return rc;
        }
        HIPCHK(hipEventSynchronize(G.ev_h[j & 1]));
        const double2* hs = G.slot(j);
        std::copy(hs, hs + hh1.size(), hh1.begin());
        std::copy(hs + hh1.size(), hs + 2 * hh1.size(), hh2.begin());
        std::memcpy(hn.data(), hs + 2 * hh1.size(), ncol * sizeof(double));
        ++total;
        bool any_active = false;
        for (int k = 0; k < ncol; ++k) {
          if (!active[k]) continue;
          for (int i = 0; i <= j; ++i) {
            const double2 a = hh1[(size_t)k * (m + 1) + i], bb = hh2[(size_t)k * (m + 1) + i];
            Hc(k, i, j) = zc(a.x + bb.x, a.y + bb.y);
          }
          Hc(k, j + 1, j) = hn[k];
          double* csk = &cs[(size_t)k * m];
          zc* snk = &sn[(size_t)k * m];
          for (int i = 0; i < j; ++i) {
            const zc t = csk[i] * Hc(k, i, j) + snk[i] * Hc(k, i + 1, j);
            Hc(k, i + 1, j) = -std::conj(snk[i]) * Hc(k, i, j) + csk[i] * Hc(k, i + 1, j);
            Hc(k, i, j) = t;
          }
          givens(Hc(k, j, j), Hc(k, j + 1, j), csk[j], snk[j]);
          Hc(k, j, j) = csk[j] * Hc(k, j, j) + snk[j] * Hc(k, j + 1, j);
          Hc(k, j + 1, j) = 0.0;
          zc* ek = &e1[(size_t)k * (m + 1)];
          ek[j + 1] = -std::conj(snk[j]) * ek[j];
          ek[j] = csk[j] * ek[j];
          jc[k] = j + 1;
          col_iters[k] += 1;
          const double est = std::abs(ek[j + 1]) / bnorm[k];
          if (k == 0) hist.push_back(est);
          if (est <= o.tol || hn[k] == 0.0 || std::abs(Hc(k, j, j)) == 0.0) active[k] = 0;
          any_active |= active[k];
        }
        if (!any_active) {
          ++j;
          break;
        }
      }
    } else {
      // Delayed reorthogonalisation: step j returns a^(j) = V_{<j}^H x_j and nu_j (x_j =
      // nu_j v_j + V_{<j} a^(j)) together with c^(j) = V_{<=j}^H w_j and s_j = |w_j|, where
      // x_{j+1} = (w_j - V_{<=j} c^(j)) / s_j.  Hence (I - S) z_j = w_j = V_{<=j} (c^(j) + s_j a^(j+1))
      // + s_j nu_{j+1} v_{j+1}: Hessenberg column j is complete once step j + 1 has run.  The
      // host stops on a provisional column j (its subdiagonal from Pythagoras, without the delayed
      // correction) and then completes it from step j + 1, which is already queued: no more
      // steps run than with the undelayed form.
      const int kmax = std::min(m, o.maxit - total);  // columns of this cycle; step kmax only closes it
      auto launch_dstep = [&](int jj) -> int {
        int r2 = (jj < kmax) ? arnoldi_step(c, S, G, jj) : arnoldi_kernels_dcgs(c, S, G, jj, true);
        if (r2) return r2;
        HIPCHK(hipEventRecord(G.ev_h[jj & 1], c->st));
        return HBJ_OK;
      };
      rc = launch_dstep(0);
      if (rc) return rc;
      bool stop_next = false;
      std::vector<zc> hp(m + 2);
      for (int j = 0;; ++j) {
        if (!stop_next && j + 1 <= kmax) {
          rc = launch_dstep(j + 1);
          if (rc) return rc;
        }
        HIPCHK(hipEventSynchronize(G.ev_h[j & 1]));
        const double2* hs = G.slot(j);
        const double2* ha = hs;
        const double2* hcv = hs + (size_t)ncol * (m + 1);
        const double* hsc = (const double*)(hs + 2 * (size_t)ncol * (m + 1));
        bool any_active = false;
        for (int k = 0; k < ncol; ++k) {
          if (!active[k]) continue;
          const double nu = hsc[4 * k], sj = hsc[4 * k + 1], wwj = hsc[4 * k + 2];
          const double2* ak = ha + (size_t)k * (m + 1);
          if (j < kmax) {  // x_j is a search direction: column j of R
            Rc(k, j, j) = nu;
            for (int i = 0; i < j; ++i) Rc(k, i, j) = zc(ak[i].x, ak[i].y);
          }
          zc* ek = &e1[(size_t)k * (m + 1)];
          if (j == 0) {
            ek[0] = rnorm[k] * nu;
          } else {
            const int jm = j - 1;  // complete column j - 1
            for (int i = 0; i < j; ++i) Hc(k, i, jm) = cprev[(size_t)k * (m + 1) + i] + sprev[k] * zc(ak[i].x, ak[i].y);
            const double hn = sprev[k] * nu;
            Hc(k, j, jm) = hn;
            double* csk = &cs[(size_t)k * m];
            zc* snk = &sn[(size_t)k * m];
            for (int i = 0; i < jm; ++i) {
              const zc t = csk[i] * Hc(k, i, jm) + snk[i] * Hc(k, i + 1, jm);
              Hc(k, i + 1, jm) = -std::conj(snk[i]) * Hc(k, i, jm) + csk[i] * Hc(k, i + 1, jm);
              Hc(k, i, jm) = t;
            }
            givens(Hc(k, jm, jm), Hc(k, j, jm), csk[jm], snk[jm]);
            Hc(k, jm, jm) = csk[jm] * Hc(k, jm, jm) + snk[jm] * Hc(k, j, jm);
            Hc(k, j, jm) = 0.0;
            ek[j] = -std::conj(snk[jm]) * ek[jm];
            ek[jm] = csk[jm] * ek[jm];
            jc[k] = j;
            col_iters[k] += 1;
            const double est = std::abs(ek[j]) / bnorm[k];
            if (k == 0) hist.push_back(est);
            if (est <= o.tol || hn == 0.0 || std::abs(Hc(k, jm, jm)) == 0.0) active[k] = 0;
          }
          for (int i = 0; i <= j; ++i) {
            const double2 cv = hcv[(size_t)k * (m + 1) + i];
            cprev[(size_t)k * (m + 1) + i] = zc(cv.x, cv.y);
          }
          sprev[k] = sj;
          wwprev[k] = wwj;
          any_active |= active[k];
        }
        if (j >= 1) ++total;
        if (j == kmax || !any_active) break;
        if (stop_next) {
          // The provisional column j - 1 met the tolerance but the completed one did not (the
          // delayed correction raised its subdiagonal): the cycle goes on.  Step j + 1 was not
          // queued ahead, so it is launched now.
          stop_next = false;
          rc = launch_dstep(j + 1);
          if (rc) return rc;
        }
        // provisional column j
        bool all_done = true;
        for (int k = 0; k < ncol && all_done; ++k) {
          if (!active[k]) continue;
          double cc = 0.0;
          for (int i = 0; i <= j; ++i) {
            hp[i] = cprev[(size_t)k * (m + 1) + i];
            cc += std::norm(hp[i]);
          }
          hp[j + 1] = std::sqrt(std::max(wwprev[k] - cc, 0.0));
          const double* csk = &cs[(size_t)k * m];
          const zc* snk = &sn[(size_t)k * m];
          for (int i = 0; i < j; ++i) {
            const zc t = csk[i] * hp[i] + snk[i] * hp[i + 1];
            hp[i + 1] = -std::conj(snk[i]) * hp[i] + csk[i] * hp[i + 1];
            hp[i] = t;
          }
          double csp;
          zc snp;
          givens(hp[j], hp[j + 1], csp, snp);
          if (std::abs(snp) * std::abs(e1[(size_t)k * (m + 1) + j]) / bnorm[k] > o.tol) all_done = false;
        }
        if (all_done) stop_next = true;
      }
    }
    // y = H^{-1} e1 per column, x += Z y (or P^{-1} V y)
    int jmax = 0;
    std::fill(yh.begin(), yh.end(), mk(0.0, 0.0));
    for (int k = 0; k < ncol; ++k) {
      if (col_conv[k] || jc[k] == 0) continue;
      const int jj = jc[k];
      std::vector<zc> y(jj);
      const zc* ek = &e1[(size_t)k * (m + 1)];
      for (int i = jj - 1; i >= 0; --i) {
        zc acc = ek[i];
        for (int l = i + 1; l < jj; ++l) acc -= Hc(k, i, l) * y[l];
        y[i] = acc / Hc(k, i, i);
      }
      if (dcgs && !G.flexible) {
        // the search directions were x_j = V R e_j: x += P^{-1} V (R y)
        std::vector<zc> ry(jj, zc(0.0));
        for (int i = 0; i < jj; ++i)
          for (int l = i; l < jj; ++l) ry[i] += Rc(k, i, l) * y[l];
        y.swap(ry);
      }
      for (int i = 0; i < jj; ++i) yh[(size_t)k * (m + 1) + i] = mk(y[i].real(), y[i].imag());
      jmax = std::max(jmax, jj);
    }
    if (jmax > 0) {
      HIPCHK(hipMemcpyAsync(G.ydev, yh.data(), yh.size() * sizeof(double2), hipMemcpyHostToDevice, c->st));
      if (G.flexible) {
        HIPCHK(launch_update(G.x, G.Z, vs, jmax, G.ydev, m + 1, mk(1.0, 0.0), nif, ncol, c->st));
      } else {
        HIPCHK(launch_fill_zero(G.w, vs * sizeof(double2), c->st));
        HIPCHK(launch_update(G.w, G.V, vs, jmax, G.ydev, m + 1, mk(1.0, 0.0), nif, ncol, c->st));
        rc = precond(c, S, G.w, G.zt, ncol);
        if (rc) return rc;
        HIPCHK(launch_axpby(G.x, G.zt, mk(1.0, 0.0), mk(1.0, 0.0), vs, c->st));
      }
    }
    // true residual
    rc = op_apply(c, S, G.x, G.w);
    if (rc) return rc;
    HIPCHK(launch_copy(G.r, G.b, vs, c->st));
    HIPCHK(launch_axpby(G.r, G.w, mk(-1.0, 0.0), mk(1.0, 0.0), vs, c->st));
    rc = G.norms(G.r, rnorm);
    if (rc) return rc;
    for (int k = 0; k < ncol; ++k) {
      if (col_conv[k]) continue;
      col_relres[k] = rnorm[k] / bnorm[k];
      if (col_relres[k] <= o.tol) col_conv[k] = 1;
    }
  }
  (void)stats;
  return HBJ_OK;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* hbj_last_error(void) { return g_last_error.c_str(); }

const char* hbj_strerror(int code) {
  switch (code) {
    case HBJ_OK: return "ok";
    case HBJ_EINVAL: return "invalid argument";
    case HBJ_ESTATE: return "call out of order";
    case HBJ_EHIP: return "HIP runtime error";
    case HBJ_EWAIT: return "dataflow dependency wait exceeded its limit";
    case HBJ_EIO: return "tuning cache file could not be written";
    case HBJ_ENOMEM: return "out of device memory";
    case HBJ_ZERO_PIVOT: return "exactly singular local matrix";
    case HBJ_NOT_CONVERGED: return "GMRES did not converge";
    default: return "unknown code";
  }
}

// (a, b) of the second-order transmission condition d_n u - i alpha a u - (i b / alpha) d_tt u = g:
// a = 1 + 0.2 i, b = 0.15 exp(-i pi / 4) (chosen by a sweep of block-Jacobi GMRES iterations on the
// 5-point grid at 10 and 15 points per wavelength; the Taylor values (1, 1/2) let S expand the
// grid-scale tangential modes)
static const double2 kTransA = {1.0, 0.2};
static const double2 kTransB = {0.15 * 0.70710678118654752, -0.15 * 0.70710678118654752};

// Pade transmission (paper Sec. 7): N_pade auxiliary fields, branch-cut rotation phi
static const int kPadeTerms = 8;
static const double kPadePhi = 1.04719755119659774615;  // pi / 3

// order of the band's transmission closure: the Pade form factors the Robin-closed matrices
// and corrects them in the dense operators
static int transmission_order(const hbj_ctx* c) { return c->P.transmission == 2 ? 2 : 1; }

static int assemble_medium(hbj_ctx* c) {
  Geom& g = c->g;
  const int order = transmission_order(c);
  const double2 ta = order == 2 ? kTransA : mk(1.0, 0.0), tb = order == 2 ? kTransB : mk(0.0, 0.0);
  HIPCHK(launch_if_coef(g, c->m, c->pos_tab, ta, c->coef, c->st));
  HIPCHK(launch_if_band(g, c->m, c->pos_tab, order, ta, tb, c->coef, c->band, c->st));
  HIPCHK(launch_local_diag(g, c->m, c->ft, c->coef, c->band, c->diag, c->st));
  c->factored = false;
  return HBJ_OK;
}

int hbj_setup(const hbj_problem* prob, const double* c_dev, void* stream, hbj_ctx** out) {
  if (!prob || !out || !c_dev) return fail(HBJ_EINVAL, "null argument");
  *out = nullptr;
  const hbj_problem& P = *prob;
  if (P.nx < 2 || P.ny < 2 || P.n1 < 1 || P.n2 < 1 || P.nx % P.n1 || P.ny % P.n2)
    return fail(HBJ_EINVAL, "grid must be divisible by the decomposition");
  if (P.nx / P.n1 < 2 || P.ny / P.n2 < 2) return fail(HBJ_EINVAL, "subdomains must be at least 2 x 2");
  if (P.nx / P.n1 > 256) return fail(HBJ_EINVAL, "subdomain width above 256 is not supported");
  if (!(P.k >= 0.0) || !std::isfinite(P.k)) return fail(HBJ_EINVAL, "k must be finite and >= 0");
  if (P.precision != HBJ_FP64 && P.precision != HBJ_MIXED) return fail(HBJ_EINVAL, "bad precision");
  if (P.precond < HBJ_PC_NONE || P.precond > HBJ_PC_BJ) return fail(HBJ_EINVAL, "bad preconditioner");
  if (P.bj_combine < 0 || P.bj_combine > 1 || P.bj_compose < 0 || P.bj_compose > 1 || P.bj_width < 0)
    return fail(HBJ_EINVAL, "bad block-Jacobi option");
  if (P.operator_form != HBJ_OP_BANDED && P.operator_form != HBJ_OP_DENSE)
    return fail(HBJ_EINVAL, "bad operator form");
  if (P.sweep_exec != HBJ_SWEEP_DATAFLOW && P.sweep_exec != HBJ_SWEEP_STEPPED)
    return fail(HBJ_EINVAL, "bad sweep execution option");
  if (P.transmission < 0 || P.transmission > 3) return fail(HBJ_EINVAL, "transmission must be 0, 1, 2 or 3");
  if (P.transmission == 3 && P.operator_form != HBJ_OP_DENSE)
    return fail(HBJ_EINVAL, "the Pade transmission needs the dense operator form");
  if (P.operator_form == HBJ_OP_DENSE && 2 * (P.nx / P.n1 + P.ny / P.n2) > 1024)
    return fail(HBJ_EINVAL, "dense operators need 2 (sub_nx + sub_ny) <= 1024");
  if ((size_t)P.nx * P.ny > (size_t)1 << 31) return fail(HBJ_EINVAL, "grid too large");
  std::unique_ptr<hbj_ctx> c(new hbj_ctx());
  c->P = P;
  c->st = (hipStream_t)stream;
  HIPCHK(hipGetDevice(&c->dev));
  HIPCHK(volume_residual_scratch_init(c->dev));
  {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, c->dev));
    c->arch = prop.gcnArchName;
    c->arch = c->arch.substr(0, c->arch.find(':'));  // gfx950 from gfx950:sramecc+:xnack-
    for (char& ch : c->arch)
      if (!std::isalnum((unsigned char)ch)) ch = '_';
  }
  Geom& g = c->g;
  g.nx = P.nx;
  g.ny = P.ny;
  g.n1 = P.n1;
  g.n2 = P.n2;
  g.snx = P.nx / P.n1;
  g.sny = P.ny / P.n2;
  g.nloc = g.snx * g.sny;
  g.kl = g.ku = g.snx;
  g.kv = g.kl + g.ku;
  g.ldab = 2 * g.kl + g.ku + 1;
  g.h = (P.h > 0.0) ? P.h : 1.0 / (P.nx + 1);
  g.k = P.k;
  c->ndom = P.n1 * P.n2;
  c->ne = 2 * P.n1 * P.n2 - P.n1 - P.n2;
  c->ng = P.n1 + P.n2 - 1;
  if (P.precond == HBJ_PC_SGS) c->bj_width = std::max(1, c->ng - 1);
  else c->bj_width = (P.bj_width > 0) ? P.bj_width : P.n1;
  if (c->ng >= 2) build_blocks(c.get());
  std::vector<int32_t> pos_tab;
  build_layout(c.get(), pos_tab);
  SolveLayout& L = c->L;
  L.nb = 16;
  L.nblk = (g.nloc + L.nb - 1) / L.nb;
  L.wf = L.nb + g.kl;
  L.mf_per_sub = (size_t)L.nblk * L.nb * L.wf;
  L.pf_per_sub = (size_t)L.nblk * L.wf;
  set_backward_window(c.get(), g.kv);
  // additive reading: the shared groups (start of every forward interval but the first;
  // top of every backward interval but the first)
  std::vector<int32_t> rf, rb;
  for (size_t b = 1; b < c->fblocks.size(); ++b) {
    const int a = c->fblocks[b].first;
    rf.push_back(c->grp_lo[a]);
    rf.push_back(c->grp_hi[a]);
  }
  for (size_t b = 1; b < c->bblocks.size(); ++b) {
    const int a = c->bblocks[b].second;
    rb.push_back(c->grp_lo[a]);
    rb.push_back(c->grp_hi[a]);
  }
  c->nranges_f = (int)rf.size() / 2;
  c->nranges_b = (int)rb.size() / 2;
  const size_t npts = (size_t)g.nx * g.ny;
  int* bad = nullptr;
  if (dalloc(&c->ft, c->ndom) || dalloc(&c->coef, (size_t)g.nif) || dalloc(&c->band, (size_t)g.nif) ||
      dalloc(&c->pos_tab, pos_tab.size()) ||
      dalloc(&c->m, npts) || dalloc(&c->diag, (size_t)c->ndom * g.nloc) || dalloc(&c->ranges_f, rf.size()) ||
      dalloc(&c->ranges_b, rb.size()) || dalloc(&c->info, (size_t)c->ndom) || dalloc(&bad, 1))
    return fail(HBJ_ENOMEM, "setup allocation failed");
  HIPCHK(hipMemcpyAsync(c->ft, c->ft_host.data(), c->ndom * sizeof(FaceTab), hipMemcpyHostToDevice, c->st));
  if (!pos_tab.empty())
    HIPCHK(hipMemcpyAsync(c->pos_tab, pos_tab.data(), pos_tab.size() * 4, hipMemcpyHostToDevice, c->st));
  if (!rf.empty()) HIPCHK(hipMemcpyAsync(c->ranges_f, rf.data(), rf.size() * 4, hipMemcpyHostToDevice, c->st));
  if (!rb.empty()) HIPCHK(hipMemcpyAsync(c->ranges_b, rb.data(), rb.size() * 4, hipMemcpyHostToDevice, c->st));
  HIPCHK(launch_fill_zero(bad, 4, c->st));
  HIPCHK(launch_check_medium(c_dev, (int)npts, bad, c->st));
  int nbad = 0;
  HIPCHK(hipMemcpyAsync(&nbad, bad, 4, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  dfree(bad);
  if (nbad) return fail(HBJ_EINVAL, "wave speed must be finite and positive");
  HIPCHK(launch_c_to_m(c_dev, c->m, (int)npts, c->st));
  int rc = assemble_medium(c.get());
  if (rc) return rc;
  if (P.operator_form == HBJ_OP_DENSE) {
    // row blocks of the stepped launches (forward, backward, every face)
    std::vector<int32_t> rbl;
    const int masks[3] = {kMaskFwd, kMaskBwd, 0xF};
    const int Lif = local_if_len(g);
    for (int i = 0; i < 3; ++i) {
      c->rbl_off[i] = (int)rbl.size();
      for (int rb = 0; rb * kTR < Lif; ++rb) {
        bool use = false;
        for (int row = rb * kTR; row < std::min(Lif, rb * kTR + kTR); ++row) {
          int f, e;
          local_if_face(g, row, &f, &e);
          use |= ((masks[i] >> f) & 1) != 0;
        }
        if (use) rbl.push_back(rb);
      }
      c->rbl_n[i] = (int)rbl.size() - c->rbl_off[i];
    }
    c->rbl_host = rbl;
    if (dalloc(&c->rbl, rbl.size()) || dalloc(&c->df_err, 1)) return fail(HBJ_ENOMEM, "setup allocation failed");
    HIPCHK(hipMemcpyAsync(c->rbl, rbl.data(), rbl.size() * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(launch_fill_zero(c->df_err, sizeof(int32_t), c->st));
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    c->df_grid = std::max(1, ncu) * sweep_df_occupancy(Lif, P.precision == HBJ_MIXED);
  }
  HIPCHK(hipEventCreate(&c->ev0));
  HIPCHK(hipEventCreate(&c->ev1));
  HIPCHK(hipStreamSynchronize(c->st));
  *out = c.release();
  return HBJ_OK;
}

int hbj_set_slowness2(hbj_ctx* c, const double* m_dev) {
  if (!c || !m_dev) return fail(HBJ_EINVAL, "null argument");
  const size_t npts = (size_t)c->g.nx * c->g.ny;
  // validate through c = m^{-1/2} > 0: reuse the positivity check on m directly
  int* bad = nullptr;
  HIPCHK(dalloc(&bad, 1));
  HIPCHK(launch_fill_zero(bad, 4, c->st));
  HIPCHK(launch_check_medium(m_dev, (int)npts, bad, c->st));
  int nbad = 0;
  HIPCHK(hipMemcpyAsync(&nbad, bad, 4, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  dfree(bad);
  if (nbad) return fail(HBJ_EINVAL, "squared slowness must be finite and positive");
  HIPCHK(hipMemcpyAsync(c->m, m_dev, npts * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  return assemble_medium(c);
}

// Dense scattering operators: one unit-datum local solve per (subdomain, interface
// position), in chunks, then T_s[row][col] = -sigma x_row - rho delta_{row,col} (row blocks).
// The Pade form's dense operators (after the unit-datum solves with the Robin-closed factors have
// filled W = A_b^-1 U): face blocks on the host, then G^-1 = (I + C U^T W)^-1 and
// T = -P - Sigma U^T W G^-1 J on the device.
static int build_pade(hbj_ctx* c) {
  const Geom& g = c->g;
  if (!c->Wl) return fail(HBJ_ENOMEM, "the Pade transmission needs the dense lifting matrices (device memory)");
  const int L = local_if_len(g);
  const size_t fbs = pade_fb_per_sub(g), nfb = fbs * c->ndom;
  std::vector<double> mh((size_t)g.nx * g.ny);
  std::vector<IfCoef> ch((size_t)std::max(g.nif, 1));
  HIPCHK(hipMemcpyAsync(mh.data(), c->m, mh.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(ch.data(), c->coef, (size_t)g.nif * sizeof(IfCoef), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  std::vector<double2> hP(nfb), hS(nfb), hJ(nfb), hC(nfb);
  if (pade_face_blocks(g, c->ft_host.data(), mh.data(), ch.data(), kPadeTerms, kPadePhi, hP.data(), hS.data(),
                       hJ.data(), hC.data()))
    return fail(HBJ_ZERO_PIVOT, "singular face matrix I/h - (i/2) X of the Pade transmission");
  const size_t nG = (size_t)c->ndom * L * L;
  if (!c->pade_P) {
    if (dalloc(&c->pade_P, nfb) || dalloc(&c->pade_S, nfb) || dalloc(&c->pade_J, nfb) || dalloc(&c->pade_C, nfb) ||
        dalloc(&c->Ginv, nG))
      return fail(HBJ_ENOMEM, "Pade operator allocation failed");
  }
  HIPCHK(hipMemcpyAsync(c->pade_P, hP.data(), nfb * sizeof(double2), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->pade_S, hS.data(), nfb * sizeof(double2), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->pade_J, hJ.data(), nfb * sizeof(double2), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->pade_C, hC.data(), nfb * sizeof(double2), hipMemcpyHostToDevice, c->st));
  double2* work = nullptr;
  int32_t* piv = nullptr;
  int32_t* info = nullptr;
  if (dalloc(&work, 2 * nG) || dalloc(&piv, (size_t)c->ndom * L) || dalloc(&info, (size_t)c->ndom)) {
    dfree(work);
    dfree(piv);
    return fail(HBJ_ENOMEM, "Pade workspace allocation failed");
  }
  hipError_t he = launch_pade_T(g, c->ft, c->Wl, c->pade_P, c->pade_S, c->pade_J, c->pade_C, c->Ginv, work, piv, info,
                                c->T64, c->st);
  std::vector<int32_t> ih(c->ndom);
  if (he == hipSuccess) he = hipMemcpyAsync(ih.data(), info, c->ndom * sizeof(int32_t), hipMemcpyDeviceToHost, c->st);
  if (he == hipSuccess) he = hipStreamSynchronize(c->st);
  dfree(work);
  dfree(piv);
  dfree(info);
  if (he != hipSuccess) return fail(HBJ_EHIP, std::string("Pade operators: ") + hipGetErrorString(he));
  for (int s = 0; s < c->ndom; ++s)
    if (ih[s]) {
      c->zero_sub = s;
      c->zero_row = ih[s] - 1;
      return fail(HBJ_ZERO_PIVOT, "singular Woodbury matrix I + C M of the Pade form in subdomain " +
                                      std::to_string(s));
    }
  return HBJ_OK;
}

static int build_dense(hbj_ctx* c) {
  const Geom& g = c->g;
  const int L = local_if_len(g);
  const size_t per = t_per_sub(g);
  if (!c->T64 && dalloc(&c->T64, per * c->ndom)) return fail(HBJ_ENOMEM, "dense operator allocation failed");
  if (c->P.precision == HBJ_MIXED && !c->T32 && dalloc(&c->T32, per * c->ndom))
    return fail(HBJ_ENOMEM, "dense operator allocation failed");
  // dense lifting operators when memory allows (else the lifting stays banded)
  if (!c->Wl && dalloc(&c->Wl, (size_t)c->ndom * g.nloc * L) != hipSuccess) {
    c->Wl = nullptr;
    (void)hipGetLastError();
  }
  if (c->Wl) HIPCHK(launch_fill_zero(c->Wl, (size_t)c->ndom * g.nloc * L * sizeof(double2), c->st));
  HIPCHK(launch_fill_zero(c->T64, per * c->ndom * sizeof(double2), c->st));
  std::vector<Entry> all;
  for (int s = 0; s < c->ndom; ++s)
    for (int col = 0; col < L; ++col) {
      int f, ee;
      local_if_face(g, col, &f, &ee);
      if (c->ft_host[s].in_off[f] >= 0) all.push_back(Entry{s, col, 0, 0});
    }
  const int chunk = (int)std::min<size_t>(4096, all.size());
  Entry* dev = nullptr;
  int2* tdev = nullptr;
  HIPCHK(dalloc(&dev, (size_t)chunk));
  if (dalloc(&tdev, (size_t)chunk) != hipSuccess) {
    dfree(dev);
    return fail(HBJ_ENOMEM, "dense operator workspace allocation failed");
  }
  SolveIO io{};
  io.unit = 1;
  int rc = HBJ_OK;
  for (size_t off = 0; off < all.size() && rc == HBJ_OK; off += chunk) {
    const int n = (int)std::min<size_t>(chunk, all.size() - off);
    std::vector<int2> tiles;
    append_tiles(all, off, n, tiles);
    hipError_t he = hipMemcpyAsync(dev, all.data() + off, n * sizeof(Entry), hipMemcpyHostToDevice, c->st);
    if (he == hipSuccess)
      he = hipMemcpyAsync(tdev, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, c->st);
    if (he != hipSuccess) { rc = fail(HBJ_EHIP, hipGetErrorString(he)); break; }
    rc = run_solves<double>(c, dev, n, io, tdev, (int)tiles.size());
    if (rc) break;
    he = launch_build_T(g, dev, n, c->ft, c->band, (const double2*)c->ybuf, (size_t)c->L.nblk * c->L.nb, c->T64,
                        c->st);
    if (he == hipSuccess && c->Wl)
      he = launch_build_W(g, dev, n, c->ft, c->coef, (const double2*)c->ybuf, (size_t)c->L.nblk * c->L.nb, c->Wl,
                          c->st);
    if (he != hipSuccess) rc = fail(HBJ_EHIP, hipGetErrorString(he));
  }
  hipError_t he = hipStreamSynchronize(c->st);
  dfree(dev);
  dfree(tdev);
  if (rc) return rc;
  if (he != hipSuccess) return fail(HBJ_EHIP, hipGetErrorString(he));
  if (is_pade(c)) {
    rc = build_pade(c);
    if (rc) return rc;
  }
  if (c->T32) HIPCHK(launch_cast_c64(c->T64, c->T32, per * c->ndom, c->st));
  return HBJ_OK;
}

int hbj_factor(hbj_ctx* c) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  c->graph_epoch++;  // captured iterations refer to the operators being rebuilt
  const Geom& g = c->g;
  const SolveLayout& L = c->L;
  const size_t nband = (size_t)c->ndom * g.nloc * g.ldab;
  const size_t mb_full = (size_t)L.nblk * L.nb * (L.nb + g.kv);  // the backward window with interchanges
  if (!c->ab) {
    if (dalloc(&c->ab, nband) || dalloc(&c->ipiv, (size_t)c->ndom * g.nloc) ||
        dalloc(&c->mf64, L.mf_per_sub * c->ndom) || dalloc(&c->mb64, mb_full * c->ndom) ||
        dalloc(&c->pf, L.pf_per_sub * c->ndom) || dalloc(&c->pflag, (size_t)L.nblk * c->ndom))
      return fail(HBJ_ENOMEM, "factor allocation failed");
    if (c->P.precision == HBJ_MIXED &&
        (dalloc(&c->mf32, L.mf_per_sub * c->ndom) || dalloc(&c->mb32, mb_full * c->ndom)))
      return fail(HBJ_ENOMEM, "factor allocation failed");
  }
  c->factored = false;
  {
    ProfScope ps(c, HBJ_K_FACTOR, (double)nband * 16.0, 8.0 * c->ndom * (double)g.nloc * g.kl * g.kv);
    HIPCHK(launch_band_assemble(g, c->diag, c->ft, c->band, c->ab, c->ndom, c->st));
    HIPCHK(launch_band_lu(g, c->ab, c->ipiv, c->info, c->ndom, c->st));
  }
  std::vector<int32_t> info(c->ndom);
  HIPCHK(hipMemcpyAsync(info.data(), c->info, c->ndom * 4, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  c->zero_sub = c->zero_row = -1;
  for (int s = 0; s < c->ndom; ++s)
    if (info[s]) {
      c->zero_sub = s;
      c->zero_row = info[s] - 1;
      return fail(HBJ_ZERO_PIVOT, "exactly zero pivot in subdomain " + std::to_string(s) + " row " +
                                      std::to_string(info[s] - 1));
    }
  if (c->P.operator_form == HBJ_OP_BANDED) {
    // row interchanges anywhere?  Without any, the backward window holds only the ku rows of U's band.
    // The dense form keeps the full window: with the short one its single-source solve measured 2.5%
    // slower on the same device (same kernel durations, longer gaps between the sweep-step launches),
    // for 0.02 s less factorisation
    std::vector<int32_t> ip((size_t)c->ndom * g.nloc);
    HIPCHK(hipMemcpyAsync(ip.data(), c->ipiv, ip.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    bool swaps = false;
    for (size_t k = 0; k < ip.size() && !swaps; ++k) swaps = ip[k] != (int32_t)(k % (size_t)g.nloc);
    set_backward_window(c, swaps ? g.kv : g.ku);
  }
  HIPCHK(launch_repack(g, L, c->ab, c->ipiv, c->mf64, c->pf, c->pflag, c->mb64, c->ndom, c->st));
  {  // blocks with row interchanges anywhere (the MFMA solves skip the permutation step without them)
    std::vector<int32_t> fl((size_t)L.nblk * c->ndom);
    HIPCHK(hipMemcpyAsync(fl.data(), c->pflag, fl.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    c->interchanges = std::find(fl.begin(), fl.end(), 0) != fl.end();
  }
  if (c->P.precision == HBJ_MIXED) {
    HIPCHK(launch_cast_c64(c->mf64, c->mf32, L.mf_per_sub * c->ndom, c->st));
    HIPCHK(launch_cast_c64(c->mb64, c->mb32, L.mb_per_sub * c->ndom, c->st));
  }
  c->dense = false;
  if (c->P.operator_form == HBJ_OP_DENSE && c->g.nif > 0) {
    const int rc = build_dense(c);
    if (rc) return rc;
    c->dense = true;
  }
  HIPCHK(hipStreamSynchronize(c->st));
  c->factored = true;
  return HBJ_OK;
}

int hbj_zero_pivot(const hbj_ctx* c, int32_t* subdomain, int32_t* row) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (subdomain) *subdomain = c->zero_sub;
  if (row) *row = c->zero_row;
  return HBJ_OK;
}

int hbj_apply_operator(hbj_ctx* c, const hbj_c128* g, hbj_c128* out, int32_t nrhs) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nrhs < 1 || !g || !out) return fail(HBJ_EINVAL, "bad arguments");
  Schedule* S;
  rc = build_schedule(c, nrhs, &S);
  if (rc) return rc;
  rc = op_apply(c, S, (const double2*)g, (double2*)out);
  if (rc == HBJ_OK && (df_enabled(c, S) || c->part_err)) rc = df_check(c);
  return rc;
}

int hbj_apply_preconditioner(hbj_ctx* c, const hbj_c128* r, hbj_c128* z, int32_t nrhs) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nrhs < 1 || !r || !z) return fail(HBJ_EINVAL, "bad arguments");
  Schedule* S;
  rc = build_schedule(c, nrhs, &S);
  if (rc) return rc;
  rc = precond(c, S, (const double2*)r, (double2*)z, nrhs);
  if (rc == HBJ_OK && (df_enabled(c, S) || c->part_err)) rc = df_check(c);
  return rc;
}

int hbj_lifting(hbj_ctx* c, const hbj_c128* f, hbj_c128* b, int32_t nrhs) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nrhs < 1 || !f || !b) return fail(HBJ_EINVAL, "bad arguments");
  Schedule* S;
  rc = build_schedule(c, nrhs, &S);
  if (rc) return rc;
  if (c->g.nif == 0) return HBJ_OK;
  rc = run_lifting(c, S, (const double2*)f, (double2*)b, nrhs);
  if (rc == HBJ_OK && c->part_err) rc = part_check(c);
  return rc;
}

int hbj_reconstruct(hbj_ctx* c, const hbj_c128* f, const hbj_c128* g, hbj_c128* u, int32_t nrhs) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nrhs < 1 || !f || !u) return fail(HBJ_EINVAL, "bad arguments");
  Schedule* S;
  rc = build_schedule(c, nrhs, &S);
  if (rc) return rc;
  rc = run_reconstruct(c, S, (const double2*)f, (const double2*)g, (double2*)u, nrhs, false);
  if (rc == HBJ_OK && c->part_err) rc = part_check(c);
  return rc;
}

static int solve_impl(hbj_ctx* c, const double2* f, double2* u, int nrhs, const hbj_solve_opts* opts,
                      hbj_solve_stats* stats) {
  auto t0 = std::chrono::steady_clock::now();
  hbj_solve_opts o{1e-6, 50, 1000, 1};
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.restart < 1 || o.maxit < 0 || (o.flexible != 0 && o.flexible != 1))
    return fail(HBJ_EINVAL, "bad solve options");
  // flexible = 1 keeps the preconditioned search directions (FGMRES storage): with a fixed
  // preconditioner the iterates are those of right-preconditioned GMRES, and the solution update
  // is one pass over them.  flexible = 0 stores only the Krylov basis and applies the
  // preconditioner once more to the combination of basis vectors at the end of each cycle.
  Schedule* S;
  int rc = build_schedule(c, nrhs, &S);
  if (rc) return rc;
  const int64_t ls0 = c->local_solves;
  c->ir_max = 0;
  c->ir_resid_max = 0.0;
  std::vector<int> iters;
  std::vector<double> relres, hist;
  std::vector<char> conv;
  if (c->g.nif == 0) {  // one subdomain: the lifting is the solution
    SolveIO io{};
    io.f = f;
    io.u = u;
    rc = run_solves<double>(c, S->dev + S->all_first, S->all_count, io, S->tiles + S->all_tile_first, S->all_tile_count);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(c->st));
    iters.assign(nrhs, 0);
    relres.assign(nrhs, 0.0);
    conv.assign(nrhs, 1);
    hist.assign(1, 0.0);
  } else {
    if (!c->gm || !c->gm->matches(S, nrhs, c->g.nif, o.restart, o.flexible != 0)) {
      destroy_gmres(c->gm);
      c->gm = new Gmres();
      c->gm->c = c;
      c->gm->S = S;
      c->gm->ncol = nrhs;
      c->gm->nif = c->g.nif;
      c->gm->m = o.restart;
      c->gm->flexible = o.flexible != 0;
      rc = c->gm->alloc();
      if (rc) {
        destroy_gmres(c->gm);
        c->gm = nullptr;
        return rc;
      }
    }
    Gmres& G = *c->gm;
    rc = ensure_pc(c, nrhs);  // every buffer an iteration uses exists before any capture
    if (rc) return rc;
    rc = run_lifting(c, S, f, G.b, nrhs);
    if (rc) return rc;
    const bool forked = c->Wl != nullptr;
    if (forked) {
      rc = fork_source_part(c, S, f, u);
      if (rc) return rc;
    }
    rc = gmres_solve(c, S, G, o, stats, iters, relres, conv, hist);
    if (rc) {
      if (forked) (void)hipStreamSynchronize(c->side);
      return rc;
    }
    rc = run_reconstruct(c, S, f, G.x, u, nrhs, forked);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(c->st));
  }
  int nconv = 0, itmax = 0;
  double rmax = 0.0;
  for (int k = 0; k < nrhs; ++k) {
    nconv += conv[k] ? 1 : 0;
    itmax = std::max(itmax, iters[k]);
    rmax = std::max(rmax, relres[k]);
  }
  if (stats) {
    stats->iters = itmax;
    stats->steps_per_pc = hbj_steps_per_preconditioner(c);
    stats->local_ir_max = (c->P.precision == HBJ_MIXED) ? c->ir_max : 0;
    stats->local_ir_resid = (c->P.precision == HBJ_MIXED) ? c->ir_resid_max : 0.0;
    stats->converged = nconv;
    stats->relres = rmax;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->local_solves = (c->local_solves - ls0) / std::max(1, nrhs);
    if (stats->res_hist) {
      const int nh = std::min<int>(stats->res_hist_len, (int)hist.size());
      for (int i = 0; i < nh; ++i) stats->res_hist[i] = hist[i];
      stats->res_hist_len = nh;
    } else {
      stats->res_hist_len = 0;
    }
  }
  return (nconv == nrhs) ? HBJ_OK : HBJ_NOT_CONVERGED;
}

int hbj_solve(hbj_ctx* c, const hbj_c128* f, hbj_c128* u, int32_t nrhs, const hbj_solve_opts* opts,
              hbj_solve_stats* stats) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nrhs < 1 || !f || !u || (const void*)f == (const void*)u) return fail(HBJ_EINVAL, "bad arguments");
  rc = solve_impl(c, (const double2*)f, (double2*)u, nrhs, opts, stats);
  if (rc >= 0) {
    const int rw = df_check(c);
    if (rw) return rw;
  }
  return rc;
}

int hbj_gradient(hbj_ctx* c, const hbj_c128* f, int32_t nsrc, const int32_t* rec_idx, int32_t nrec,
                 const hbj_c128* d, double* grad_m, double* loss, hbj_c128* u_out, const hbj_solve_opts* opts,
                 hbj_solve_stats* stats) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nsrc < 1 || nrec < 1 || !f || !rec_idx || !d || !grad_m || !loss) return fail(HBJ_EINVAL, "bad arguments");
  const Geom& g = c->g;
  const int npts = g.nx * g.ny;
  std::vector<int32_t> rec(nrec);
  HIPCHK(hipMemcpyAsync(rec.data(), rec_idx, nrec * 4, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  {
    std::vector<int32_t> sr(rec);
    std::sort(sr.begin(), sr.end());
    if (sr.front() < 0 || sr.back() >= npts || std::adjacent_find(sr.begin(), sr.end()) != sr.end())
      return fail(HBJ_EINVAL, "receiver indices must be distinct nodes of the grid");
  }
  double2 *u = nullptr, *fa = nullptr, *mu = nullptr, *res = nullptr;
  auto cleanup = [&]() {
    if (!u_out) dfree(u);
    dfree(fa);
    dfree(mu);
    dfree(res);
  };
  if ((!u_out && dalloc(&u, (size_t)nsrc * npts)) || dalloc(&fa, (size_t)nsrc * npts) ||
      dalloc(&mu, (size_t)nsrc * npts) || dalloc(&res, (size_t)nsrc * nrec)) {
    cleanup();
    return fail(HBJ_ENOMEM, "gradient workspace allocation failed");
  }
  if (u_out) u = (double2*)u_out;
  hbj_solve_stats s1{}, s2{};
  rc = solve_impl(c, (const double2*)f, u, nsrc, opts, &s1);
  if (rc < 0) { cleanup(); return rc; }
  int rc_fwd = rc;
  hipError_t he = launch_gather_receivers(u, rec_idx, nrec, npts, (const double2*)d, res, nsrc, c->st);
  if (he == hipSuccess) he = launch_fill_zero(fa, (size_t)nsrc * npts * sizeof(double2), c->st);
  if (he == hipSuccess) he = launch_spread_adjoint(res, rec_idx, nrec, npts, fa, nsrc, c->st);
  if (he != hipSuccess) { cleanup(); return fail(HBJ_EHIP, hipGetErrorString(he)); }
  std::vector<double2> rh((size_t)nsrc * nrec);
  he = hipMemcpyAsync(rh.data(), res, rh.size() * sizeof(double2), hipMemcpyDeviceToHost, c->st);
  if (he == hipSuccess) he = hipStreamSynchronize(c->st);
  if (he != hipSuccess) { cleanup(); return fail(HBJ_EHIP, hipGetErrorString(he)); }
  double L = 0.0;
  for (const double2& v : rh) L += v.x * v.x + v.y * v.y;
  *loss = 0.5 * L;
  rc = solve_impl(c, fa, mu, nsrc, opts, &s2);
  if (rc < 0) { cleanup(); return rc; }
  he = launch_grad_accumulate(g, c->m, u, mu, nsrc, grad_m, c->st);
  if (he == hipSuccess) he = hipStreamSynchronize(c->st);
  cleanup();
  if (he != hipSuccess) return fail(HBJ_EHIP, hipGetErrorString(he));
  const int rw = df_check(c);
  if (rw) return rw;
  if (stats) {
    *stats = s1;
    stats->iters = std::max(s1.iters, s2.iters);
    stats->relres = std::max(s1.relres, s2.relres);
    stats->seconds = s1.seconds + s2.seconds;
    stats->converged = std::min(s1.converged, s2.converged);
  }
  return (rc_fwd == HBJ_OK && rc == HBJ_OK) ? HBJ_OK : HBJ_NOT_CONVERGED;
}

int hbj_volume_residual(hbj_ctx* c, const hbj_c128* f, const hbj_c128* u, int32_t nrhs, double* relres) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (nrhs < 1 || !f || !u || !relres) return fail(HBJ_EINVAL, "bad arguments");
  const int nblk = volume_residual_blocks(c->g);
  if ((size_t)nrhs > c->vr_cap) {
    dfree(c->vr_part);
    c->vr_part = nullptr;
    c->vr_cap = 0;
    // partial pairs of every workgroup, then the nrhs totals
    if (dalloc(&c->vr_part, (size_t)nrhs * (2 * nblk + 2))) return fail(HBJ_ENOMEM, "residual workspace allocation failed");
    c->vr_cap = nrhs;
  }
  double* sums = c->vr_part + (size_t)nrhs * 2 * nblk;
  HIPCHK(launch_volume_residual(c->g, c->m, (const double2*)f, (const double2*)u, nrhs, c->vr_part, sums, c->st));
  std::vector<double> h(2 * (size_t)nrhs);
  HIPCHK(hipMemcpyAsync(h.data(), sums, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  for (int k = 0; k < nrhs; ++k) relres[k] = h[2 * k + 1] > 0 ? std::sqrt(h[2 * k] / h[2 * k + 1]) : std::sqrt(h[2 * k]);
  return HBJ_OK;
}

int hbj_volume_residual_noalloc(hbj_ctx* c, const hbj_c128* f, const hbj_c128* u, int32_t nrhs, double* relres) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (!f || !u || !relres) return fail(HBJ_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > HBJ_VR_NOALLOC_MAX_RHS)
    return fail(HBJ_EINVAL, "nrhs must be between 1 and HBJ_VR_NOALLOC_MAX_RHS (" +
                                std::to_string(HBJ_VR_NOALLOC_MAX_RHS) + ") for the allocation-free residual");
  const hipError_t e = launch_volume_residual_noalloc(c->dev, c->g, c->m, (const double2*)f, (const double2*)u, nrhs,
                                                      relres, c->st);
  if (e == hipErrorNotInitialized) return fail(HBJ_ESTATE, "scratch of the context's device not resolved");
  if (e != hipSuccess) return fail(HBJ_EHIP, std::string("volume residual launch: ") + hipGetErrorString(e));
  return HBJ_OK;
}

int hbj_local_solve(hbj_ctx* c, int32_t nbatch, const int32_t* sub_host, const hbj_c128* rhs, hbj_c128* x,
                    int32_t precision) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (nbatch < 1 || !sub_host || !rhs || !x) return fail(HBJ_EINVAL, "bad arguments");
  if (precision == HBJ_MIXED && !c->mf32) return fail(HBJ_EINVAL, "context has no complex64 factors");
  if (is_pade(c))
    return fail(HBJ_EINVAL, "the Pade form factors the Robin-closed local matrices; its local solves are not exposed");
  std::vector<Entry> ent(nbatch);
  for (int i = 0; i < nbatch; ++i) {
    if (sub_host[i] < 0 || sub_host[i] >= c->ndom) return fail(HBJ_EINVAL, "subdomain index out of range");
    ent[i] = Entry{sub_host[i], 0, 0, 0};
  }
  Entry* dev = nullptr;
  HIPCHK(dalloc(&dev, nbatch));
  HIPCHK(hipMemcpyAsync(dev, ent.data(), nbatch * sizeof(Entry), hipMemcpyHostToDevice, c->st));
  SolveIO io{};
  io.rhs64 = (const double2*)rhs;
  io.x64 = (double2*)x;
  if (precision == HBJ_MIXED) rc = run_solves<float>(c, dev, nbatch, io);
  else rc = run_solves<double>(c, dev, nbatch, io);
  hipError_t he = hipStreamSynchronize(c->st);
  dfree(dev);
  if (rc) return rc;
  if (he != hipSuccess) return fail(HBJ_EHIP, hipGetErrorString(he));
  return HBJ_OK;
}

int hbj_band_factors(hbj_ctx* c, int32_t s, hbj_c128* ab, int32_t* ipiv) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (s < 0 || s >= c->ndom || !ab || !ipiv) return fail(HBJ_EINVAL, "bad arguments");
  const size_t nb = (size_t)c->g.nloc * c->g.ldab;
  HIPCHK(hipMemcpyAsync(ab, c->ab + (size_t)s * nb, nb * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
  HIPCHK(hipMemcpyAsync(ipiv, c->ipiv + (size_t)s * c->g.nloc, c->g.nloc * 4, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return HBJ_OK;
}

int32_t hbj_interface_len(const hbj_ctx* c) { return c ? c->g.nif : -1; }

int hbj_sizes(const hbj_ctx* c, int32_t* sub_nx, int32_t* sub_ny, int32_t* n_loc, int32_t* kl, int32_t* ndom) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (sub_nx) *sub_nx = c->g.snx;
  if (sub_ny) *sub_ny = c->g.sny;
  if (n_loc) *n_loc = c->g.nloc;
  if (kl) *kl = c->g.kl;
  if (ndom) *ndom = c->ndom;
  return HBJ_OK;
}

int32_t hbj_steps_per_preconditioner(const hbj_ctx* c) {
  if (!c) return -1;
  if (c->P.precond == HBJ_PC_NONE || c->ndom == 1) return 0;
  int f = 0, b = 0;
  for (auto& x : c->fblocks) f = std::max(f, x.second - x.first);
  for (auto& x : c->bblocks) b = std::max(b, x.second - x.first);
  return f + b;
}

int hbj_set_profiling(hbj_ctx* c, int32_t on) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  c->prof = on != 0;
  return HBJ_OK;
}

int hbj_kernel_stats(hbj_ctx* c, int32_t k, hbj_kernel_stat* out) {
  if (!c || !out || k < 0 || k >= HBJ_K_NCLASS) return fail(HBJ_EINVAL, "bad arguments");
  *out = c->ks[k];
  return HBJ_OK;
}

int hbj_set_sweep_wait(hbj_ctx* c, int32_t max_polls, int32_t stall_task) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  c->df_spin = max_polls > 0 ? max_polls : kDfSpinDefault;
  c->df_stall = stall_task >= 0 ? stall_task : -1;
  return HBJ_OK;
}

int hbj_set_graphs(hbj_ctx* c, int32_t on) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  c->use_graphs = on != 0;
  return HBJ_OK;
}

int hbj_set_orthogonalization(hbj_ctx* c, int32_t mode) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (mode != HBJ_ORTH_CGS2 && mode != HBJ_ORTH_DCGS2 && mode != HBJ_ORTH_SSTEP && mode != HBJ_ORTH_AUTO)
    return fail(HBJ_EINVAL, "unknown orthogonalisation");
  if (mode != c->orth) ++c->graph_epoch;  // the captured steps hold the other kernels
  c->orth = mode;
  return HBJ_OK;
}

int hbj_set_step_chaining(hbj_ctx* c, int32_t on) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (on != 0 && on != 1) return fail(HBJ_EINVAL, "step chaining must be 0 or 1");
  c->chain_ok = on != 0;
  return HBJ_OK;
}

int hbj_set_sstep_block(hbj_ctx* c, int32_t s) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (s < 1 || s > kSstepMax) return fail(HBJ_EINVAL, "s-step block out of range");
  c->sstep_block = s;
  return HBJ_OK;
}

int hbj_set_multi_solve(hbj_ctx* c, int32_t mode) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (mode != HBJ_MSOLVE_CHAINS && mode != HBJ_MSOLVE_MFMA) return fail(HBJ_EINVAL, "unknown multi-solve mode");
  if (mode != c->msolve) ++c->graph_epoch;  // the captured steps hold the other kernels
  c->msolve = mode;
  return HBJ_OK;
}

int hbj_set_operator_overlap(hbj_ctx* c, int32_t on) {
  if (!c || (on != 0 && on != 1)) return fail(HBJ_EINVAL, "bad arguments");
  c->op_overlap = on != 0;
  return HBJ_OK;
}

int hbj_set_solve_tuning(hbj_ctx* c, int32_t shape) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  if (shape < -1 || shape >= kSolveShapes) return fail(HBJ_EINVAL, "solve launch shape out of range");
  c->solve_shape_fixed = shape;
  return HBJ_OK;
}

int hbj_set_solve_partitions(hbj_ctx* c, int32_t np) {
  if (!c || np < 0 || np == 1 || np > 4096) return fail(HBJ_EINVAL, "bad run count");
  c->part_np = np == 0 ? kPartDefault : np;
  return HBJ_OK;
}

int hbj_get_solve_tuning(const hbj_ctx* c, int32_t* n, char* keys, int32_t* shapes, float* us) {
  if (!c || !n || *n < 0) return fail(HBJ_EINVAL, "bad arguments");
  const int cap = *n;
  int i = 0;
  for (const auto& kv : c->solve_choice) {
    if (i < cap) {
      if (keys) {
        std::strncpy(keys + (size_t)i * 96, kv.first.c_str(), 95);
        keys[(size_t)i * 96 + 95] = 0;
      }
      if (shapes) shapes[i] = kv.second.shape;
      if (us)
        for (int v = 0; v < kSolveShapes; ++v) us[(size_t)i * kSolveShapes + v] = kv.second.us[v];
    }
    ++i;
  }
  *n = i;
  return HBJ_OK;
}

int hbj_get_tuning(const hbj_ctx* c, int32_t* variants, float* us) {
  if (!c || !variants) return fail(HBJ_EINVAL, "bad arguments");
  for (int i = 0; i < 4; ++i) {
    variants[i] = c->mm_variant[i];
    if (us)
      for (int v = 0; v < kMmVariants; ++v) us[i * kMmVariants + v] = c->mm_us[i][v];
  }
  return HBJ_OK;
}

int hbj_set_tuning(hbj_ctx* c, const int32_t* variants) {
  if (!c || !variants) return fail(HBJ_EINVAL, "bad arguments");
  for (int i = 0; i < 4; ++i)
    if (variants[i] < -1 || variants[i] >= kMmVariants) return fail(HBJ_EINVAL, "tuning variant out of range");
  for (int i = 0; i < 4; ++i) {
    c->mm_variant[i] = variants[i];
    for (int v = 0; v < kMmVariants; ++v) c->mm_us[i][v] = 0.f;
  }
  return HBJ_OK;
}

int hbj_reset_kernel_stats(hbj_ctx* c) {
  if (!c) return fail(HBJ_EINVAL, "null context");
  for (auto& k : c->ks) k = hbj_kernel_stat{};
  return HBJ_OK;
}

void hbj_destroy(hbj_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  delete c;
}

}  // extern "C"
