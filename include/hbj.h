/*
 * hbj.h - C ABI of the MI355X (gfx950) block-Jacobi sweeping preconditioner for
 * the 2-D Helmholtz equation (R. Dai, "A Block Jacobi Sweeping Preconditioner
 * for the Helmholtz Equation", arXiv 2209.10886).
 *
 * Problem (paper Sec. 3, eq. (1)): (-Lap - k^2 m) u = f on the unit square with
 * the first-order absorbing condition (d_n - i alpha) u = 0 on the outer boundary,
 * m = 1/c^2, time dependence e^{-i omega t}.  Discretisation: 5-point finite
 * differences on an nx x ny interior grid, nodes ((ix+1) h, (iy+1) h), with a
 * Robin face template (u_q - u_p)/h - i alpha (u_p + u_q)/2 = g imposed at each
 * face midpoint; alpha = k sqrt(m_p) on outer faces and k sqrt((m_p + m_q)/2) on
 * interfaces.
 *
 * Method: a non-overlapping n1 x n2 checkerboard (Sec. 2) with Robin
 * transmission conditions (Sec. 3, eq. (2)); GMRES on the interface system
 * (I - S) g = b (Sec. 4, eq. (5)), right-preconditioned by the SGS sweeping
 * preconditioner (Sec. 5, eq. (7)) or the block-Jacobi sweeping preconditioner
 * (Sec. 6); every local problem is solved with a batched banded LU on the GPU.
 *
 * Conventions (all entry points):
 *  - Array arguments are DEVICE pointers, read and written in stream order on the
 *    stream given to hbj_setup.  The caller owns every buffer it passes; the
 *    library owns the factors and its workspace (allocated by hbj_setup and
 *    hbj_factor, freed by hbj_destroy).
 *  - Fields (c, m, f, u, gradients) are [ny][nx] row-major (x fastest); a batch of
 *    nrhs fields is [nrhs][ny][nx].
 *  - Interface vectors (g, b, residuals) are in the paper's m order (Sec. 2,
 *    Definitions 1-2): block m(i, j) holds the data subdomain i RECEIVES from its
 *    neighbour j; blocks on vertical interfaces hold sub_ny entries ordered by
 *    increasing y, blocks on horizontal interfaces sub_nx entries ordered by
 *    increasing x.  A batch is [nrhs][n_if] with n_if = hbj_interface_len().
 *  - hbj_c128 is {double re, im}, the memory layout of torch.complex128.
 *  - Return codes: 0 on success; negative = error (nothing useful was written);
 *    positive = numerical outcome (outputs are written).  hbj_last_error() gives
 *    a message for the last failure on the calling thread.
 *  - A context is not thread-safe; use one context per stream.
 */
#ifndef HBJ_H
#define HBJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbj_ctx hbj_ctx;
typedef struct { double re, im; } hbj_c128;

/* return codes */
enum {
  HBJ_OK = 0,
  HBJ_EINVAL = -1,         /* bad size, option, pointer or non-finite medium   */
  HBJ_ESTATE = -2,         /* call out of order (e.g. solve before factor)     */
  HBJ_EHIP = -3,           /* a HIP runtime call failed                        */
  HBJ_ENOMEM = -4,         /* device allocation failed                         */
  HBJ_EWAIT = -5,          /* a dataflow sweep's dependency wait exceeded its
                              poll limit; the outputs of the call are invalid  */
  HBJ_EIO = -6,            /* the tuning cache file could not be written       */
  HBJ_ZERO_PIVOT = 1,      /* exactly singular local matrix (see hbj_factor)   */
  HBJ_NOT_CONVERGED = 2    /* GMRES hit maxit; outputs hold the last iterate   */
};

/* precision of the subdomain factors */
enum { HBJ_FP64 = 0,       /* complex128 factors everywhere                      */
       HBJ_MIXED = 1 };    /* complex64 factors: preconditioner in complex64, the
                              operator's local solves refined to FP64 accuracy
                              (iterative refinement with an FP64 residual),
                              flexible GMRES, Arnoldi and residuals in FP64     */
/* preconditioner */
enum { HBJ_PC_NONE = 0, HBJ_PC_SGS = 1, HBJ_PC_BJ = 2 };
/* how block-Jacobi intervals combine at their shared anti-diagonal group */
enum { HBJ_BJ_RESTRICTED = 0,   /* upstream interval owns the shared group        */
       HBJ_BJ_ADDITIVE = 1 };   /* both contributions summed (literal Sec. 6 sum) */
/* how the scattering operators are applied inside GMRES */
enum { HBJ_OP_BANDED = 0,       /* a banded local solve per application (Sec. 4)   */
       HBJ_OP_DENSE = 1 };      /* each subdomain's local scattering operator formed
                                   once as a dense L x L matrix (L = 2 sub_nx +
                                   2 sub_ny) at factor time; every application is
                                   then a batched matrix-vector product           */
/* how the sweep steps of the dense form are launched */
enum { HBJ_SWEEP_STEPPED = 0,   /* one launch per sweep step (Sec. 5-6 order)     */
       HBJ_SWEEP_DATAFLOW = 1 };/* one launch per preconditioner application (plus
                                   the operator inside GMRES): tasks = row blocks
                                   of (subdomain, right-hand side), each waiting
                                   only on the tasks that produce its data.  The
                                   hand-off between tasks costs several device-
                                   coherent memory round trips per step, more than
                                   a launch boundary on MI355X, so this form is
                                   slower; kept as an option and for comparison  */
/* how the forward and backward block-Jacobi passes compose */
enum { HBJ_BJ_PRODUCT = 0,      /* z = B_U^{-1} B_L^{-1} r, like SGS              */
       HBJ_BJ_RESIDUAL = 1 };   /* additive-projection half steps (Sec. 6)        */

typedef struct {
  int32_t nx, ny;        /* interior grid; both divisible by the decomposition      */
  double  h;             /* grid spacing; 0 selects 1/(nx+1)                        */
  double  k;             /* reference wavenumber (kappa = k sqrt(m))                */
  int32_t n1, n2;        /* checkerboard: n1 columns (x), n2 rows (y), Sec. 2       */
  int32_t precision;     /* HBJ_FP64 | HBJ_MIXED                                    */
  int32_t precond;       /* HBJ_PC_NONE | HBJ_PC_SGS | HBJ_PC_BJ                    */
  int32_t bj_width;      /* anti-diagonals per partial sweep; 0 = n1 (Sec. 6)      */
  int32_t bj_combine;    /* HBJ_BJ_RESTRICTED | HBJ_BJ_ADDITIVE                     */
  int32_t bj_compose;    /* HBJ_BJ_PRODUCT | HBJ_BJ_RESIDUAL                        */
  int32_t operator_form; /* HBJ_OP_BANDED | HBJ_OP_DENSE                            */
  int32_t sweep_exec;    /* HBJ_SWEEP_STEPPED | HBJ_SWEEP_DATAFLOW (dense form, fewer
                            than 4 right-hand sides; identical results up to the
                            order of floating-point sums)                         */
  int32_t transmission;  /* order of the transmission condition on interface faces:
                            0 or 1 = the Robin condition (d_n - i alpha) u = g;
                            2 = second order, d_n u - i alpha a u - (i b / alpha)
                            d_tt u = g with a = 1 + 0.2 i, b = 0.15 exp(-i pi/4)
                            (the paper's condition is a higher-order absorbing
                            one, Sec. 7; the tangential term follows a second-order
                            expansion of the one-way operator, with coefficients
                            that damp the grid-scale modes).  The outer faces keep
                            the absorbing condition, so the solution does not
                            depend on it.  Any operator form; in the banded form the
                            traces follow the solves in a second kernel;
                            3 = the Pade condition of the paper's experiments (Sec. 7:
                            8 auxiliary fields, branch rotation pi/3): the impedance
                            becomes the dense symmetric face matrix K^1/2 R(D) K^1/2,
                            R the rotated Pade approximation of sqrt(1 + D), D the
                            tangential second difference of the face (Neumann face
                            ends), K the interface wavenumbers.  Dense operator form
                            only (HBJ_EINVAL otherwise): the band factors keep the
                            Robin closure and the operators, lifting and
                            reconstruction are corrected on the edge nodes by a
                            Woodbury identity; hbj_local_solve is not available   */
} hbj_problem;

typedef struct {
  double  tol;           /* stop at ||b - (I-S) g|| <= tol ||b|| (Sec. 7: 1e-6)     */
  int32_t restart;       /* GMRES restart length (50)                               */
  int32_t maxit;         /* total iteration cap                                     */
  int32_t flexible;      /* 1: flexible GMRES, the preconditioned search directions
                            z_j = P^{-1} v_j are kept and the solution update is
                            x += Z y (the mixed-precision form, whose complex64
                            preconditioner is applied inside an FP64 FGMRES);
                            0: GMRES, only the Krylov basis is kept and x +=
                            P^{-1} (V y), one more preconditioner application per
                            restart cycle.  With a fixed preconditioner both give
                            the same iterates (up to rounding); 1 moves less data.
                            Default (opts = NULL): 1.  Other values: HBJ_EINVAL  */
} hbj_solve_opts;

typedef struct {
  int32_t iters;         /* GMRES iterations (max over right-hand sides)            */
  int32_t steps_per_pc;  /* sequential sweep steps per preconditioner application  */
  int32_t local_ir_max;  /* HBJ_MIXED with banded operators: most complex64 solves
                            spent on one refined local solve of the operator (1 +
                            refinement steps); 0 otherwise                        */
  int32_t converged;     /* number of right-hand sides that reached tol             */
  double  relres;        /* max over right-hand sides of the final true residual    */
  double  seconds;       /* wall time of the call                                   */
  int64_t local_solves;  /* subdomain solves performed (per right-hand side)        */
  double* res_hist;      /* caller-owned HOST buffer or NULL: Givens residual
                            estimates relative to ||b|| of right-hand side 0,
                            entry 0 = 1.0                                          */
  int32_t res_hist_len;  /* capacity of res_hist on input, entries written on output */
  double  local_ir_resid;/* HBJ_MIXED with banded operators: largest relative residual
                            ||rhs - A_s x|| / ||rhs|| (FP64) left by a refined local
                            solve; refinement stops at 1e-14 or when a step no longer
                            halves it (at most 8 solves).  A value far above
                            eps64 cond(A_s) flags a local problem too ill-conditioned
                            for complex64 factors; 0 otherwise                   */
} hbj_solve_stats;

typedef struct {         /* per kernel class, accumulated while profiling is on     */
  int64_t launches;
  double  ms;            /* summed kernel time between HIP events on the stream (the
                            dense single-launch classes use the dispatch's own start
                            and stop times)                                        */
  double  bytes;         /* summed algorithmic bytes (factor entries + vectors)     */
  double  flops;         /* summed algorithmic flops                                */
} hbj_kernel_stat;

/* kernel classes for hbj_kernel_stats */
enum { HBJ_K_FWD = 0, HBJ_K_BWD = 1, HBJ_K_FACTOR = 2, HBJ_K_KRYLOV = 3, HBJ_K_SCATTER = 4,
       HBJ_K_SWEEP = 5,     /* dataflow sweep launches (HBJ_SWEEP_DATAFLOW)      */
       HBJ_K_LIFT = 6,      /* dense lifting and reconstruction products         */
       HBJ_K_OPERATOR = 7,  /* dense operator (I - S) applications; HBJ_K_SCATTER
                               then counts the preconditioner's sweep steps      */
       HBJ_K_NCLASS = 8 };

/*
 * hbj_setup - describe the problem and build the decomposition (paper Secs. 2-3).
 *   prob    host pointer, copied.
 *   c_dev   device [ny][nx] float64 wave speed c > 0, finite; m = 1/c^2 is kept.
 *   stream  hipStream_t (as void*) on which every later call of the context runs;
 *           NULL = the null stream.
 *   out     receives the new context.
 * Assembles the local operators A_i (5-point stencil + Robin faces, eq. (2)) in
 * LAPACK band storage (kl = ku = sub_nx).  Errors: HBJ_EINVAL for sizes not
 * divisible by n1 / n2, subdomains smaller than 2 x 2, a non-finite or
 * non-positive c, or unknown options; HBJ_ENOMEM.
 */
int hbj_setup(const hbj_problem* prob, const double* c_dev, void* stream, hbj_ctx** out);

/*
 * hbj_set_slowness2 - replace the medium by m = 1/c^2 directly (device [ny][nx]
 * float64, finite, > 0).  Invalidates the factors (hbj_factor must run again).
 */
int hbj_set_slowness2(hbj_ctx* ctx, const double* m_dev);

/*
 * hbj_factor - batched banded LU with partial pivoting of every local matrix
 * (the paper's "sparse direct solver" of the sub-problems, Sec. 7), LAPACK
 * zgbtrf semantics (pivot = first max of |re| + |im|), followed by the repack
 * into the blocked solve layout and, for HBJ_MIXED, the rounding to complex64.
 * With HBJ_OP_BANDED, when no local factorisation interchanged a row, U keeps the
 * ku superdiagonals of A and the backward solves carry only those (the kl further
 * superdiagonals that interchanges can fill are zero); otherwise, and in the dense
 * form, they carry kl + ku.  Returns HBJ_ZERO_PIVOT if some U(j,j) is exactly zero (the factors are then
 * unusable); hbj_zero_pivot() reports the first (subdomain, row).
 */
int hbj_factor(hbj_ctx* ctx);
int hbj_zero_pivot(const hbj_ctx* ctx, int32_t* subdomain, int32_t* row);

/*
 * hbj_apply_operator - out = (I - S) g for nrhs interface vectors (Sec. 4, eq. (5)):
 * one local solve per subdomain with its incoming data as Robin data, then the
 * outgoing traces -rho g - sigma u written into the receivers' blocks.
 *   g, out  device [nrhs][n_if] hbj_c128; may not alias.
 */
int hbj_apply_operator(hbj_ctx* ctx, const hbj_c128* g, hbj_c128* out, int32_t nrhs);

/*
 * hbj_apply_preconditioner - z = P^{-1} r with the context's preconditioner:
 * SGS (Sec. 5, eq. (7)) or block Jacobi (Sec. 6; intervals of bj_width
 * anti-diagonals swept concurrently in lockstep).  PC_NONE copies r.
 *   r, z    device [nrhs][n_if] hbj_c128; may not alias.
 */
int hbj_apply_preconditioner(hbj_ctx* ctx, const hbj_c128* r, hbj_c128* z, int32_t nrhs);

/*
 * hbj_lifting - b = outgoing traces of the lifting w_i (Sec. 4, eq. (3)):
 * local solves with the source and zero transmission data.  In the dense form
 * (HBJ_OP_DENSE, when the n_loc x L lifting operators fit in memory) each
 * subdomain with a nonzero source is one matrix-vector product with the rows of
 * A_i^{-1} at its edge nodes, taken from the unit-datum solves of hbj_factor.
 *   f device [nrhs][ny][nx], b device [nrhs][n_if].
 */
int hbj_lifting(hbj_ctx* ctx, const hbj_c128* f, hbj_c128* b, int32_t nrhs);

/*
 * hbj_reconstruct - u_i = A_i^{-1}(f_i + B_i g) on every subdomain (Sec. 4).
 *   f, u device [nrhs][ny][nx]; g device [nrhs][n_if].
 */
int hbj_reconstruct(hbj_ctx* ctx, const hbj_c128* f, const hbj_c128* g, hbj_c128* u, int32_t nrhs);

/*
 * hbj_solve - u = A^{-1} f for nrhs sources by the interface problem of the
 * decomposition: the lifting b (Sec. 4, eq. (3)), the interface system
 * (I - S) g = b (Sec. 4, eq. (5)) solved by right-preconditioned GMRES with restarts
 * to ||b - (I - S) g|| <= tol ||b|| (Sec. 7 solves it with GMRES to 1e-6), the
 * preconditioner of the context (Sec. 5, eq. (7), or Sec. 6), and the reconstruction
 * u_i = A_i^{-1}(f_i + B_i g) (Sec. 4).  The right-hand sides iterate in lockstep,
 * each with its own Krylov recurrence (a column stops once it meets tol).
 * Synchronises with the host once per iteration and returns after completion.
 *   f, u   device [nrhs][ny][nx] (may not alias); opts host (NULL = defaults
 *          tol 1e-6, restart 50, maxit 1000, flexible 1); stats host or NULL.
 * Errors: HBJ_ESTATE before hbj_factor; HBJ_EINVAL for nrhs < 1, tol <= 0,
 * restart < 1, maxit < 0 or flexible not 0 / 1; HBJ_ENOMEM (the Krylov workspace,
 * kept for later calls with the same sizes).  Returns HBJ_NOT_CONVERGED (u = last
 * iterate, stats filled) when maxit is reached.
 */
int hbj_solve(hbj_ctx* ctx, const hbj_c128* f, hbj_c128* u, int32_t nrhs,
              const hbj_solve_opts* opts, hbj_solve_stats* stats);

/*
 * hbj_gradient - loss L = 1/2 sum_s ||P u_s - d_s||^2 and dL/dm (m = 1/c^2) by
 * the adjoint state: forward solves A u_s = f_s, adjoint solves A mu_s =
 * conj(P^T r_s) with the same factors and preconditioner (A is complex symmetric,
 * lambda_s = conj(mu_s)), grad_p = -sum_s Re(conj(lambda_p) dA_pp/dm_p u_p).
 *   f       device [nsrc][ny][nx] sources
 *   rec_idx device [nrec] int32 flat node indices iy*nx + ix of the receivers (P)
 *   d       device [nsrc][nrec] observed data
 *   grad_m  device [ny][nx] float64, overwritten with dL/dm
 *   loss    HOST double, receives L
 *   u_out   device [nsrc][ny][nx] or NULL: the forward fields
 */
int hbj_gradient(hbj_ctx* ctx, const hbj_c128* f, int32_t nsrc, const int32_t* rec_idx, int32_t nrec,
                 const hbj_c128* d, double* grad_m, double* loss, hbj_c128* u_out,
                 const hbj_solve_opts* opts, hbj_solve_stats* stats);

/*
 * hbj_volume_residual - relative residual of the global discrete problem (Sec. 3, eq. (1)):
 * relres[k] = ||f_k - A u_k|| / ||f_k|| (||A u_k|| when f_k = 0), A the 5-point operator on the
 * whole grid with the absorbing condition on the outer faces.  It does not involve the
 * decomposition, so it measures how well a field from hbj_solve solves the original problem.
 * Needs hbj_setup only (not hbj_factor).  Synchronises with the host.
 *   f, u    device [nrhs][ny][nx] hbj_c128
 *   relres  HOST [nrhs]
 * Errors: HBJ_EINVAL (null pointers, nrhs < 1), HBJ_ENOMEM (its small reduction workspace, kept
 * for later calls), HBJ_EHIP.
 */
int hbj_volume_residual(hbj_ctx* ctx, const hbj_c128* f, const hbj_c128* u, int32_t nrhs, double* relres);

/*
 * hbj_volume_residual_noalloc - the same relative residual as hbj_volume_residual, for callers
 * that cannot allocate memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  It calls no allocating routine: the per-workgroup partial sums go to a
 * static scratch array of the library (1 MiB per device, holding up to HBJ_VR_NOALLOC_MAX_RHS
 * right-hand sides; each device holds it until the process ends), and the result stays on the
 * device.  Asynchronous: enqueued on the context's stream, no host synchronisation.
 *   f, u    device [nrhs][ny][nx] hbj_c128
 *   relres  DEVICE [nrhs] float64, written in stream order
 * Every call on one device shares that device's scratch array, which keeps the last call's
 * partial sums (each call writes every partial it reads, so nothing needs clearing): calls that
 * overlap on one device (two streams, two contexts, two host threads) race and give undefined
 * results.  Errors: HBJ_EINVAL (null pointers, nrhs < 1 or nrhs > HBJ_VR_NOALLOC_MAX_RHS; nothing
 * is enqueued), HBJ_ESTATE (the scratch address of the context's device is resolved by
 * hbj_setup; a failure there is reported by hbj_setup), HBJ_EHIP.
 */
#define HBJ_VR_NOALLOC_MAX_RHS 64
int hbj_volume_residual_noalloc(hbj_ctx* ctx, const hbj_c128* f, const hbj_c128* u, int32_t nrhs, double* relres);

/*
 * hbj_local_solve - x_e = A_{s_e}^{-1} rhs_e for a batch of subdomains (the unit
 * of work of every operator above), using the factored band.
 *   sub_host  HOST [nbatch] int32 subdomain indices s = (i2-1) n1 + (i1-1)
 *   rhs, x    device [nbatch][sub_nx*sub_ny] hbj_c128 in local order ly*sub_nx+lx.
 *   precision HBJ_FP64 or HBJ_MIXED (complex64 factors; needs a mixed context).
 */
int hbj_local_solve(hbj_ctx* ctx, int32_t nbatch, const int32_t* sub_host, const hbj_c128* rhs,
                    hbj_c128* x, int32_t precision);

/*
 * hbj_band_factors - copy the LAPACK-layout band LU of subdomain s (after
 * hbj_factor) into caller buffers: ab device [n_loc][2kl+ku+1] (column-major
 * band, A(i,j) at ab[j][kl+ku+i-j]) and ipiv device [n_loc] int32 (0-based).
 */
int hbj_band_factors(hbj_ctx* ctx, int32_t s, hbj_c128* ab, int32_t* ipiv);

/* sizes: n_if, sub_nx, sub_ny, n_loc, kl (= ku), number of subdomains */
int32_t hbj_interface_len(const hbj_ctx* ctx);
int hbj_sizes(const hbj_ctx* ctx, int32_t* sub_nx, int32_t* sub_ny, int32_t* n_loc, int32_t* kl, int32_t* ndom);

/* sequential steps of one preconditioner application and of its passes */
int32_t hbj_steps_per_preconditioner(const hbj_ctx* ctx);

/* kernel timing with HIP events on the context stream (adds events; off by default) */
int hbj_set_profiling(hbj_ctx* ctx, int32_t on);
int hbj_kernel_stats(hbj_ctx* ctx, int32_t kclass, hbj_kernel_stat* out);
int hbj_reset_kernel_stats(hbj_ctx* ctx);

/*
 * hbj_set_graphs - replay GMRES iterations as HIP graphs (default off).  With the
 * dense operators, stepped sweeps and fewer than 4 right-hand sides, each Arnoldi
 * step (preconditioner, operator and the Gram-Schmidt kernels: about 22 launches)
 * is captured once per step index into a graph on a capture stream and replayed
 * with one launch on the context stream; the results are identical.  Profiling
 * (hbj_set_profiling) runs the launches one by one.  Captured graphs are dropped
 * by hbj_factor and with the GMRES workspace (a different restart length or
 * number of right-hand sides).  Off by default: the host queues step j + 1 before it
 * reads step j back, so one-by-one launches already keep the GPU busy, and each graph
 * launch adds a gap of its own (measured: 8.22 ms against 8.64 ms per solve on the
 * 1024^2 grid of 8 x 8 subdomains).
 */
int hbj_set_graphs(hbj_ctx* ctx, int32_t on);

/*
 * Gram-Schmidt variant of the Arnoldi steps (the paper leaves the orthogonalisation of
 * its GMRES open; Sec. 7 uses GMRES(50)).  Both keep the basis orthonormal to working
 * precision; they differ in passes over the basis per step:
 *   HBJ_ORTH_CGS2   classical Gram-Schmidt applied twice: two inner-product passes and
 *                   two update passes (five launches);
 *   HBJ_ORTH_DCGS2  Gram-Schmidt with delayed reorthogonalisation (Bielich, Langou,
 *                   Thomas, Swirydowicz, Yamazaki and Boman, Parallel Computing 2022):
 *                   the second pass for step j's vector is merged into step j + 1, so
 *                   one inner-product pass and one update pass (two launches); Hessenberg
 *                   column j is completed one step later, and convergence is tested on a
 *                   provisional column so that no extra step runs.
 *   HBJ_ORTH_SSTEP  s-step cycles (Hoemmen, Communication-avoiding Krylov subspace
 *                   methods, 2010): s preconditioner and operator applications build the
 *                   Newton basis y_{i+1} = (I - S) P^{-1} y_i - y_i (shift 1) from the last
 *                   basis vector, then one inner-product pass and one update pass over the
 *                   basis make all s vectors orthonormal (block classical Gram-Schmidt with
 *                   the Pythagorean Cholesky QR, Carson, Lund, Rozloznik and Thomas, Linear
 *                   Algebra Appl. 2022): two passes per s steps instead of two per step.
 *                   Convergence is found at the exact step (the Hessenberg columns of a block
 *                   are formed one by one); the rest of that block's applications are unused.
 *                   Needs flexible GMRES (hbj_solve_opts.flexible = 1) and a restart length of
 *                   at most 63; HBJ_ORTH_DCGS2 is used otherwise.  s: hbj_set_sstep_block.
 *   HBJ_ORTH_AUTO   HBJ_ORTH_SSTEP where the Krylov vectors of all right-hand sides
 *                   together hold at least 2^20 entries (there a pass over the basis
 *                   outweighs the per-block costs: measured on MI355X, 64 right-hand sides on
 *                   the 2048^2 grid of 16 x 16 subdomains take 25% less time, while one on the
 *                   1024^2 grid and 16 on the 512^2 grid take longer), HBJ_ORTH_DCGS2
 *                   otherwise.  Default.
 * Restart lengths above 255 use HBJ_ORTH_CGS2.  A change drops captured graphs.
 * Returns HBJ_EINVAL for any other value.
 */
enum { HBJ_ORTH_CGS2 = 0, HBJ_ORTH_DCGS2 = 1, HBJ_ORTH_SSTEP = 2, HBJ_ORTH_AUTO = 3 };
int hbj_set_orthogonalization(hbj_ctx* ctx, int32_t mode);

/*
 * hbj_set_step_chaining - with 4 or more right-hand sides, the dense operators and the default
 * readings, each sweep step on the matrix-product path passes its outputs on to the tile of
 * gathered incoming data of the next step (Sec. 6: the data a step sends is what the next step
 * receives), and the other positions of every step's tile are gathered once at the start of the
 * pass, instead of one gather launch per step.  Used while the autotuner's variant for the sweep
 * steps reads gathered tiles.  The same results bit for bit.  on: 1 (default) or 0.  Returns
 * HBJ_EINVAL for any other value.
 */
int hbj_set_step_chaining(hbj_ctx* ctx, int32_t on);

/*
 * hbj_set_sstep_block - steps per block of the HBJ_ORTH_SSTEP cycles, 1..8 (default 8; the
 * last block of a restart cycle may be shorter).  Returns HBJ_EINVAL outside 1..8.
 */
int hbj_set_sstep_block(hbj_ctx* ctx, int32_t s);

/*
 * hbj_set_multi_solve - how the banded local solves (Sec. 4: every application of the
 * operator, of the preconditioner, the lifting and the reconstruction is a batch of solves
 * u = A_s^{-1} rhs) run when a batch holds many right-hand sides per subdomain:
 *   HBJ_MSOLVE_CHAINS  one workgroup per (subdomain, right-hand side), vector FMAs;
 *   HBJ_MSOLVE_MFMA    up to 16 right-hand sides of one subdomain per workgroup: each column
 *                      block of the triangular solves is one complex matrix product on the
 *                      matrix cores, and the factors are read once per 16 right-hand sides.
 *                      Used where a batch averages at least 8 right-hand sides per
 *                      subdomain (the formation of the dense operators at hbj_factor, with
 *                      one right-hand side per interface position; solves of 8 or more
 *                      sources in the banded form).  Default.
 * Both give the same solutions up to rounding.  Takes effect at the next call (the dense
 * operators: at the next hbj_factor).  A change drops captured graphs.  Returns HBJ_EINVAL
 * for any other value.
 */
enum { HBJ_MSOLVE_CHAINS = 0, HBJ_MSOLVE_MFMA = 1 };
int hbj_set_multi_solve(hbj_ctx* ctx, int32_t mode);

/*
 * hbj_set_operator_overlap - inside GMRES, apply the operator (I - S) z (Sec. 4, eq. (5)) to the
 * preconditioned vector z = P^{-1} v (Sec. 6) while the backward pass is still running: after
 * backward step k, the operator rows of the subdomains whose incoming and outgoing data of z the
 * pass has already finalised run on a second stream, and the context stream waits for them after
 * the pass.  Applies to the dense operators with fewer than 4 right-hand sides, stepped sweeps and
 * the default readings; profiled solves and captured graphs keep the operator after the pass.
 * Same results bit for bit.  on: 1 or 0 (default: measured slower on MI355X, where each wait of
 * one stream on another's event adds about 19 us, eight per GMRES iteration).  Returns
 * HBJ_EINVAL for any other value.
 */
int hbj_set_operator_overlap(hbj_ctx* ctx, int32_t on);

/*
 * hbj_get_tuning - choices of the autotuner of the many-right-hand-side operator
 * kernel (dense form, 4 or more right-hand sides).  On its first launch of each
 * kind the library times every variant on that launch's own data, writing into
 * scratch, and keeps the fastest.  Variant v < 12: tile depth (k-steps per batch
 * of loads) 2, 4, 8 for v % 3 = 0, 1, 2; incoming data gathered into tiles by a
 * separate launch first ((v % 6) < 3, its time included) or read straight from
 * the interface vector ((v % 6) >= 3); the 64 right-hand sides of a tile taken by
 * one group of four wavefronts (v < 6) or split over two groups (v >= 6).
 * Variants 12-15: two groups, each wavefront walking its k-steps over all faces
 * through a register ring of 4 (v even) or 8 (v odd) k-steps of loads in flight;
 * gathered (12, 13) or direct (14, 15).  Variants 16, 17: as 7 and 9 (gathered
 * with 4 k-steps per batch, direct with 2).  Variants 12-17 deal the tiles to the
 * XCDs so that all row tiles of one subdomain share an L2.  Variants 18-21: one
 * group of eight wavefronts splitting the k range (each A operand loaded once),
 * 2 or 4 k-steps per batch, gathered (18, 19) or direct (20, 21).
 * Timing: a warm-up round times every variant once; those within twice the best
 * time there run three more rounds, taking turns, and the lowest mean wins.  The
 * choice is stored in the tuning cache (hbj_tune_cache_path) under the device,
 * precision, launch kind, checkerboard, subdomain size and right-hand sides padded
 * to 16, 32, 64 or 128, and a later context with the same key reads it back
 * without timing.  With HBJ_TUNE=0 in the environment, or on a stream under graph
 * capture, and no cache entry: variant 15 for sweep steps and 7 for the operator,
 * untimed.
 *   variants  HOST [4]: complex128 sweep steps, complex128 operator, complex64
 *             sweep steps, complex64 operator; -1 = not tuned yet.
 *   us        HOST [4][22] or NULL: the measured microseconds per launch (the mean
 *             of three rounds, or the warm-up time for a variant that dropped out;
 *             all zero for a choice read from the cache, set, or taken untimed).
 */
int hbj_get_tuning(const hbj_ctx* ctx, int32_t* variants, float* us);

/*
 * Autotuned launch shapes of the banded local solves (Sec. 4: every application of the
 * operator, of the preconditioner, the lifting and the reconstruction in the banded form, and
 * the formation of the dense operators at hbj_factor, is a batch of local solves
 * u = A_s^{-1} rhs).  A batch runs in one of five launch shapes:
 *   0, 1, 2  one workgroup per (subdomain, right-hand side) with register prefetch depths
 *            (column blocks of the factors in flight per lane) forward/backward of 5/3, 3/2
 *            and 6/3 for complex128 factors, 8/4, 4/3 and 10/6 for complex64;
 *   3        16 right-hand sides of one subdomain per workgroup on MFMA (only for batches
 *            with many right-hand sides per subdomain and HBJ_MSOLVE_MFMA);
 *   4        each local solve split over np workgroups (hbj_set_solve_partitions), one per run
 *            of consecutive column blocks: the forward (backward) substitution is linear in the
 *            window rows it carries from one block to the next (kl rows forward, kl + ku
 *            backward), so every run but the last is first solved from a zero incoming state, a
 *            short chain over the runs recovers their true incoming states through the runs'
 *            transfer matrices (formed on the first such batch after each hbj_factor: the
 *            outgoing state for each unit incoming state; np - 2 matrices of kl^2 and of
 *            (kl + ku)^2 entries per subdomain and precision, held by the context), and every
 *            run but the first is solved again from its true state.  About twice the factor
 *            bytes of shapes 0-2, spread over np times the workgroups: for batches of few solves
 *            (a sweep step of a few subdomains), where one workgroup per solve leaves most of the
 *            device idle.  Timed only for batches of at most two right-hand sides per subdomain.
 * All give the same solutions up to rounding (shapes 0-2 bit for bit).  On the first batch of
 * each class - precision, subdomain size and band, number of solves (by powers of two) and
 * right-hand sides per subdomain (1, 2-3, 4-7, 8-15, 16) - the library times every candidate
 * on that batch's own data (writing only its solve workspace; a candidate at more than twice
 * the best time after the first round drops out), keeps the fastest, and records it in the
 * tuning cache file, so later contexts and processes reuse it without timing.  Without timing
 * (environment HBJ_TUNE=0, or inside a graph capture) a batch takes shape 3 where it averages at
 * least 8 right-hand sides per 16-wide tile, else shape 0.
 */

/*
 * hbj_set_solve_tuning - fix the launch shape of every banded solve batch of this context
 * (tests of every shape, reproducible timings): 0..4 as above (3 falls back to 0 where the MFMA
 * solves do not apply, 4 where the subdomain has fewer than two column blocks or a band wider
 * than the solve kernels' windows), or -1 to choose by timing (default).  Returns HBJ_EINVAL for
 * any other value.
 */
int hbj_set_solve_tuning(hbj_ctx* ctx, int32_t shape);

/*
 * hbj_set_solve_partitions - runs per local solve of launch shape 4 (the split solves): 2..4096,
 * or 0 for the default (16).  The count is capped by the subdomain's column blocks of 16 rows,
 * and rounded so that every run is nonempty (runs of ceil(blocks / np) blocks).  Tuning choices
 * and cache entries are kept per count.  Returns HBJ_EINVAL for 1, negative values or values
 * above 4096.
 */
int hbj_set_solve_partitions(hbj_ctx* ctx, int32_t np);

/*
 * hbj_get_solve_tuning - the choices made so far by this context, one per batch class.
 *   n        HOST in: capacity of the arrays; out: number of classes (may exceed the capacity:
 *            only the first min(capacity, number) are written).
 *   keys     HOST [capacity][96] or NULL: each class's cache key, NUL-terminated.
 *   shapes   HOST [capacity] or NULL: the chosen shape.
 *   us       HOST [capacity][5] or NULL: microseconds per candidate shape (0: not timed; the
 *            choice came from the cache file or was fixed).
 */
int hbj_get_solve_tuning(const hbj_ctx* ctx, int32_t* n, char* keys, int32_t* shapes, float* us);

/*
 * The tuning cache file (host code; no GPU is needed for these calls).  One JSON object,
 *   {"version": 1, "entries": {"<key>": {"variant": v, "us": [t0, ...]}, ...}},
 * read once per process and rewritten (merged with the file, then an atomic rename) after each
 * new decision.  Location: hbj_tune_cache_set_path, else the environment variable
 * HBJ_TUNE_CACHE ("" or "off": no file), else $XDG_CACHE_HOME/hbj/tune.json, else
 * $HOME/.cache/hbj/tune.json.  A file that does not parse counts as empty.
 *
 * hbj_tune_cache_path       the file in use ("" = none); the string stays valid until the next
 *                           call from the same thread.
 * hbj_tune_cache_set_path   use `path` from now on (NULL: the default rule above; "": no file)
 *                           and (re)read it.
 * hbj_tune_cache_lookup     1 and *variant set if `key` is cached, else 0; HBJ_EINVAL for NULL.
 * hbj_tune_cache_store      record key -> (variant, us[0..n-1]) and rewrite the file; keys are
 *                           1-200 characters of [A-Za-z0-9_.:|-], 0 <= n <= 64.  HBJ_EINVAL for
 *                           a bad key or size, HBJ_EIO if the file could not be written (the
 *                           entry is kept in memory).
 * hbj_tune_cache_size       number of entries in memory.
 */
const char* hbj_tune_cache_path(void);
int hbj_tune_cache_set_path(const char* path);
int hbj_tune_cache_lookup(const char* key, int32_t* variant);
int hbj_tune_cache_store(const char* key, int32_t variant, const float* us, int32_t n);
int32_t hbj_tune_cache_size(void);

/*
 * hbj_set_tuning - fix the variants of the many-right-hand-side operator kernel
 * instead of timing them (reproducible timings, tests of every variant).
 *   variants  HOST [4], same order as hbj_get_tuning; each in 0..21, or -1 to let
 *             the autotuner choose (or read the tuning cache) on the next launch
 *             of that kind.
 * Returns HBJ_EINVAL for a value outside -1..21 (nothing is changed then).
 */
int hbj_set_tuning(hbj_ctx* ctx, const int32_t* variants);

/*
 * hbj_set_sweep_wait - bounds of the dataflow sweeps' dependency waits, for tests
 * of the error path.  max_polls: polls of a completion counter before the wait
 * gives up (<= 0 restores the default, about a second); stall_task: index of a
 * task whose waits require one completion more than can ever happen (-1 = none),
 * so that a launch deterministically reports HBJ_EWAIT.  Every wave still exits:
 * a wait that gives up sets the error flag and the task completes with invalid
 * data.  The next call that synchronises returns HBJ_EWAIT and clears the flag.
 */
int hbj_set_sweep_wait(hbj_ctx* ctx, int32_t max_polls, int32_t stall_task);

const char* hbj_strerror(int code);
const char* hbj_last_error(void);
void hbj_destroy(hbj_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* HBJ_H */
