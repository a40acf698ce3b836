/*
 * dg.h -- C ABI of the MI355X (gfx950) implicit modal DG hot path.
 *
 * Franciolini, Fidkowski, Crivellini, "Efficient discontinuous Galerkin
 * implementations and preconditioners for implicit unsteady compressible flow
 * simulations", arXiv 1812.04789.
 *
 * Problem statement followed by this interface:
 *   semi-discrete system   M dW/dt + R(W) = 0                 (Sec. 3.1)
 *   Newton systems          K x = b,  K = a M + dR/dW          (Sec. 4 Eq. NEWTON,
 *                                                              Sec. 5.1 Eq. ODEDG;
 *                                                              the paper writes
 *                                                              K x + b = 0)
 *   matrix-free product     K v ~ a M v + (R(W+hv)-R(W))/h      (Sec. 5.1 Eq. DG-mf)
 *   p-multigrid V-cycle     Alg. 2 with subspace inheritance   (Sec. 6, 6.1)
 *   block-Jacobi smoother   element-wise PLU                   (Sec. 6.3)
 *   flexible GMRES          right preconditioned               (Sec. 6)
 *
 * Conventions (all entry points):
 *  - Vectors are FP64 DEVICE pointers owned by the caller, length dg_ndof(),
 *    layout W[element][equation][mode]: element e = i + nx*(j + ny*k) of the
 *    periodic box, equations (rho, rho u, rho v, rho w, rho e0), modes of the
 *    orthonormal Legendre tensor basis L_a(xi1) L_b(xi2) L_c(xi3),
 *    L_a(t) = sqrt((2a+1)/2) P_a(t), in hierarchical order (shell
 *    max(a,b,c), then (a,b,c) lexicographic, a most significant); the modes of
 *    degree <= q are the first (q+1)^3 of every (element, equation) run.
 *  - Every call enqueues on the context's HIP stream and returns without
 *    waiting, except fgmres_step and dg_bdf2_step (which synchronise to test
 *    convergence and fill their statistics), dg_assemble_operator (which
 *    synchronises to free its unpacked blocks) and dg_create/dg_destroy.
 *  - The context owns all internal device memory (factors, coarse operators,
 *    Krylov basis, scratch); nothing it returns must be freed by the caller.
 *  - Output vectors must not alias inputs (DG_EINVAL).
 *  - No C++ exception crosses the ABI.  On error the call returns a negative
 *    dg_status and dg_last_error() describes it.
 */
#ifndef DG_MI355X_H
#define DG_MI355X_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

typedef enum {
    DG_OK = 0,
    DG_EINVAL = -1,      /* bad argument, size, alias or mesh                  */
    DG_ENOMEM = -2,      /* device allocation failed                           */
    DG_EHIP = -3,        /* HIP runtime error                                  */
    DG_ENOCONV = -4,     /* solver did not reach its tolerance (best x kept)   */
    DG_ENONFINITE = -5,  /* NaN/Inf met in a residual or a Krylov scalar       */
    DG_ESTATE = -6       /* call order violated (e.g. pmg_apply before setup)  */
} dg_status;

enum { DG_FP64 = 0, DG_FP32 = 1, DG_BF16 = 2 };

/* Periodic structured hexahedral mesh (Sec. 3).  vtx: optional HOST array
 * [ne][8][3] of trilinear (Q1) element vertices, local vertex v = i+2j+4k at
 * reference corner (2i-1, 2j-1, 2k-1); NULL gives the straight box.  The
 * vertex copies of an element across a periodic boundary must differ by the
 * box period.  Copied at dg_create. */
typedef struct {
    int nx, ny, nz;
    double lo[3], hi[3];
    const double* vtx;
} dg_mesh_desc;

/* Gas model (Sec. 2, Eq. NS): gamma, constant viscosity mu (0 = Euler),
 * Prandtl number Pr, BR2 penalty eta_F (Sec. 3.1 Eq. visc_flux; the paper
 * requires eta_F > number of element faces). */
typedef struct {
    double gamma, mu, Pr, eta;
} dg_phys;

/* p-multigrid preconditioner (Sec. 6, Alg. 2; Sec. 6.1; Sec. 6.3).
 *  n_levels       1..4; p_level[0] must equal the context's p and the degrees
 *                 must decrease.  n_levels == 1 is the single-grid element
 *                 block-Jacobi preconditioner z = D^-1 r.
 *  nu_pre/nu_post damped block-Jacobi sweeps x += omega D^-1 (b - K x) per level.
 *  coarsest_iters right-preconditioned GMRES(BJ) iterations on the coarsest level
 *                 (1..63).
 *  prec_fine      DG_FP64 or DG_FP32: storage/arithmetic of the level-0 PLU factors.
 *  prec_coarse    DG_FP64, DG_FP32 or DG_BF16: storage of the assembled coarse
 *                 operator blocks (BF16: rounded to nearest even, products
 *                 accumulated in FP32); coarse block-Jacobi factors are FP64
 *                 for DG_FP64 and FP32 otherwise.
 *  coarse_matrix_free  how the inherited coarse operators K_l = P^T K_0 P
 *                 (Sec. 6.1) are applied: 0 = assembled for every coarse level
 *                 (diagonal + 6 face-coupling blocks per element, block-sparse
 *                 product); 1 = matrix-free for every coarse level (the
 *                 level-0 finite-difference product of Eq. DG-mf on the
 *                 zero-padded vector, then restricted); 2 = assembled on the
 *                 coarsest level only, matrix-free above it.
 *  coarsest_plain 0 = when the coarsest level is assembled with blocks of at
 *                 most 64 rows, its GMRES(BJ) runs on the right-preconditioned
 *                 operator K D^-1 stored directly (face blocks K_{e,f} X_nb,
 *                 unit diagonal; one block-sparse product per iteration, and
 *                 x = D^-1 V y at the end: the same Krylov space and iterate up
 *                 to rounding); 1 = a product with K and a block-Jacobi apply
 *                 per iteration.
 *  smoother       SMOOTH of Alg. 2 on the finer levels: 0 = nu damped
 *                 block-Jacobi sweeps; 1 = nu iterations (at most 63) of
 *                 right-preconditioned GMRES(BJ) on the residual equation,
 *                 x <- x + GMRES(K_l, D_l^-1, b - K_l x) (the smoothers of
 *                 Sec. 6, Table MGSettings: nu_pre = nu_post = 10).  omega
 *                 is not used by the GMRES smoother.
 *  cycle          0 = one V-cycle from zero (Alg. 2); 1 = the full multigrid
 *                 cycle of Alg. 1 (the level-0 right-hand side restricted to
 *                 every level, the coarsest level solved, then one V-cycle on
 *                 each finer level from the prolonged coarser result).
 *  coarsest_prec  right preconditioner of the coarsest GMRES: 0 = element
 *                 block Jacobi; 1 = block ILU(0) in minimum-discarded-fill
 *                 order (Sec. 6.3, Table MGSettings), partition-wise with the
 *                 element lines along x as partitions (couplings between
 *                 lines dropped), factors FP64, factored once per pmg_setup
 *                 (which then synchronises the stream: the elimination order
 *                 is chosen on the host).  Needs an assembled degree-1
 *                 coarsest level (n_levels >= 2, coarse_matrix_free 0 or 2). */
typedef struct {
    int n_levels;
    int p_level[4];
    int nu_pre, nu_post;
    double omega;
    int coarsest_iters;
    int prec_fine;
    int prec_coarse;
    int coarse_matrix_free;
    int coarsest_plain;
    int smoother;
    int cycle;
    int coarsest_prec;
} pmg_opts;

/* FGMRES(restart) (Sec. 6), restart 1..63: x0 = 0, converged when the recomputed true
 * residual ||b - K x|| <= rtol ||b||.  jvp_exact: 1 = tangent-linear Jacobian
 * action as the Krylov operator, 0 = the finite-difference form of Eq. DG-mf. */
typedef struct {
    int restart, max_restarts;
    double rtol;
    int jvp_exact;
} fgmres_opts;

typedef struct {
    int iters, restarts;
    double rel_res_true, rel_res_est;
} fgmres_stats;

typedef struct {
    int newton;              /* Newton iterations taken                        */
    int linear_iters;        /* FGMRES iterations summed over Newton steps     */
    double res0, res_final;  /* ||R_u(W_0)||, ||R_u(W_final)||                 */
    double max_rel_res_true; /* worst true relative linear residual           */
    double setup_seconds, solve_seconds;
} dg_step_stats;

/* Create a context for the periodic mesh, gas model and degree p (1..4) on the
 * given HIP stream (hipStream_t; NULL = default stream) of the current device.
 * Fails with DG_EINVAL on a bad mesh (non-positive Jacobian at a quadrature
 * point, n < 1), bad p or gas constants. */
dg_status dg_create(const dg_mesh_desc* mesh, const dg_phys* phys, int p, void* hip_stream, dg_ctx** out);
dg_status dg_destroy(dg_ctx* ctx);
size_t dg_ndof(const dg_ctx* ctx);                  /* ne * 5 * (p+1)^3 */
const char* dg_last_error(const dg_ctx* ctx);

/* Physical coordinates of the (p+1)^3 volume Gauss points: xyz device
 * [ne][(p+1)^3][3], points ordered (q1,q2,q3) with q3 fastest. */
dg_status dg_quad_points(dg_ctx* ctx, double* xyz);

/* L2 projection (with the volume Gauss rule) of point values given at the
 * points of dg_quad_points: values device [ne][(p+1)^3][5] -> W. */
dg_status dg_project(dg_ctx* ctx, const double* values, double* W);

/* R = R(W): volume and face integrals of Sec. 3.1 Eq. dg_ns with the Roe flux
 * and the BR2 viscous flux (Eqs. visc_flux, re). */
dg_status dg_residual(dg_ctx* ctx, const double* W, double* R);

/* y = shift * M v + (R(W + h v) - RW) / h, h = 1e-7 sqrt(1+||W||)/||v||
 * (Sec. 5.1 Eq. DG-mf; step read as scaling with 1/||v||).  RW must be R(W).
 * v = 0 gives y = 0. */
dg_status dg_jvp(dg_ctx* ctx, const double* W, const double* RW, const double* v, double shift, double* y);

/* y = shift * M v + (dR/dW)(W) v exactly (tangent-linear, forward mode). */
dg_status dg_jvp_exact(dg_ctx* ctx, const double* W, const double* v, double shift, double* y);

/* y = M v (block-diagonal mass matrix of Sec. 3.1). */
dg_status dg_mass(dg_ctx* ctx, const double* v, double* y);

/* Element diagonal blocks of K = shift M + dR/dW at W (Sec. 6.3), written to
 * the caller's device buffer blocks [ne][nb][nb], nb = 5 (p+1)^3, each block
 * COLUMN-major: blocks[e][j][i] = K[(e,i),(e,j)], local index
 * i = equation * (p+1)^3 + mode. */
dg_status dg_assemble_diag(dg_ctx* ctx, const double* W, double shift, double* blocks);

/* dg_assemble_diag without allocating: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and result as
 * dg_assemble_diag (bit for bit), but the neighbour traces it stages
 * (ne * 6 (p+1)^2 * 20 doubles) live in a fixed 128 MiB device array that the
 * library holds on every GPU it runs on until the process ends, instead of
 * context memory allocated on first use; the call makes no allocation.
 * Meshes whose traces exceed 128 MiB (above 5,592 elements at p = 4, i.e.
 * beyond 17^3; above 8,738 at p = 3, beyond 20^3) are rejected with DG_EINVAL
 * before any GPU work.  All calls
 * on one GPU share the array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller.  Enqueued on
 * the context's stream. */
dg_status dg_assemble_diag_noalloc(dg_ctx* ctx, const double* W, double shift, double* blocks);

/* Face-coupling blocks of the inherited coarse operator of degree pc
 * (Sec. 6.1, K_l = P^T K_0 P; 1 <= pc <= p, pc = p giving the face blocks of
 * the fine operator itself): off [ne][6][nbc][nbc], nbc =
 * 5 (pc+1)^3, column-major, off[e][f][j][i] = dR_{e,i}/dW_{nb(e,f),j} through
 * the integral over face f only (i, j equation-major over the modes of
 * degree <= pc).  A face whose neighbour is the element itself gives a zero
 * block (that coupling is part of the diagonal block). */
dg_status dg_assemble_coarse(dg_ctx* ctx, const double* W, int pc, double* off);

/* Matrix-based product (the assembled alternative to Eq. DG-mf that Sec. 5
 * compares against the matrix-free form): dg_assemble_operator stores
 * K = shift M + dR/dW at W, every element's diagonal block and its six
 * face-coupling blocks (7 nb^2 FP64 entries per element, held by the context
 * until the next call or dg_destroy; 23.5 GB at 16^3, p = 3; 90 GB at 16^3,
 * p = 4), and dg_jvp_assembled computes y = K v with it.
 * dg_assemble_operator assembles the blocks unpacked first, so it needs about
 * twice the held size while it runs (peak 47 GB at 16^3, p = 3), and
 * synchronises the stream before returning, when the unpacked copy is freed;
 * dg_device_bytes counts the held operator.  dg_jvp_assembled enqueues on the
 * context's stream; v and y are device [ne][5][nv], y must not alias v.
 * dg_jvp_assembled before dg_assemble_operator: DG_ESTATE. */
dg_status dg_assemble_operator(dg_ctx* ctx, const double* W, double shift);
dg_status dg_jvp_assembled(dg_ctx* ctx, const double* v, double* y);

/* Batched PLU with partial pivoting (Sec. 6.3), in place, LAPACK convention
 * (column-major blocks, rows k and piv[k] exchanged at step k, unit-lower L
 * below the diagonal).  A device [nblk][n][n], piv device int [nblk][n],
 * 1 <= n <= 625.  Enqueued on hip_stream.  A zero pivot is left in place (no
 * error). */
dg_status dg_batched_lu(void* hip_stream, double* A, int* piv, int nblk, int n);
/* x = A^-1 b for every block with the factors of dg_batched_lu; b, x device [nblk][n]. */
dg_status dg_batched_lu_solve(void* hip_stream, const double* LU, const int* piv, const double* b, double* x,
                              int nblk, int n);

/* Assemble and factor the p-multigrid preconditioner of K = shift M + dR/dW
 * at W (Sec. 6, lagged: valid until the next pmg_setup). */
dg_status pmg_setup(dg_ctx* ctx, const double* W, double shift, const pmg_opts* opts);

/* z = one V-cycle of Alg. 2 applied to r from a zero initial guess, or one
 * full multigrid cycle of Alg. 1 (pmg_opts.cycle = 1) (z ~ K^-1 r).
 * DG_ESTATE before pmg_setup. */
dg_status pmg_apply(dg_ctx* ctx, const double* r, double* z);

/* Solve K x = b by FGMRES with the current pmg preconditioner (identity if
 * pmg_setup was never called); K is linearised at W with shift given by the
 * last pmg_setup (or 0 without it).  RW must be R(W) (used by the FD
 * operator).  x is overwritten (x0 = 0).  Synchronises the stream.
 * DG_ENOCONV if max_restarts is exhausted (x holds the best iterate). */
dg_status fgmres_step(dg_ctx* ctx, const double* W, const double* RW, const double* b, double* x,
                      const fgmres_opts* opts, fgmres_stats* stats);

/* One implicit BDF2 step (Sec. 4, Eq. NEWTON with BDF2 coefficients):
 * Newton on R_u(W) = M(3W - 4Wn + Wnm1)/(2 dt) + R(W) from W_0 = Wn, linear
 * systems (3/(2dt) M + dR/dW) x = -R_u by fgmres_step with the pMG
 * preconditioner set up once at Wn (lagged over the step).  Stops when
 * ||R_u|| <= newton_rtol ||R_u(W_0)|| or ||R_u|| <= 1e-14 (3/(2dt)) ||M Wn||,
 * at most max_newton iterations (DG_ENOCONV after that).  Wnm1 == NULL means
 * Wnm1 = Wn.  Wnp1 must not alias Wn or Wnm1. */
dg_status dg_bdf2_step(dg_ctx* ctx, const double* Wn, const double* Wnm1, double dt, const pmg_opts* popts,
                       const fgmres_opts* fopts, double newton_rtol, int max_newton, double* Wnp1,
                       dg_step_stats* stats);

/* One ESDIRK3 step (Sec. 4, Eq. NEWTON): the four-stage, third-order,
 * explicit-first-stage singly diagonally implicit Runge-Kutta scheme the paper
 * uses (Kennedy & Carpenter's tableau, as in Bijl et al. 2002; stiffly
 * accurate, so Wnp1 is the last stage).  Stage 1 is Wn; stages 2..4 solve
 * M (W - Wn)/(gamma dt) + sum_{j<i} (a_ij/gamma) R(W^j) + R(W) = 0 by Newton
 * from the previous stage, linear systems (M/(gamma dt) + dR/dW) x = -R_s by
 * fgmres_step with the pMG preconditioner set up once at Wn and lagged over
 * all three implicit stages (the MFL option of Sec. 7.3).  Per stage Newton
 * stops as in dg_bdf2_step (1e-14 floor with a = 1/(gamma dt)); stats sum the
 * Newton and FGMRES iterations of the stages, res0 is the second stage's
 * initial residual and res_final the last stage's final one; DG_ENOCONV if a
 * stage did not converge.  Holds 4 more N-vectors than dg_bdf2_step. */
dg_status dg_esdirk3_step(dg_ctx* ctx, const double* Wn, double dt, const pmg_opts* popts, const fgmres_opts* fopts,
                          double newton_rtol, int max_newton, double* Wnp1, dg_step_stats* stats);

/* pmg_apply replays the V-cycle as a HIP graph captured after each
 * pmg_setup (enabled by default; the launch sequence of a V-cycle is fixed
 * by the setup).  enable = 0 runs every launch eagerly on the context stream.
 * Graph replay is skipped while per-kernel timing is enabled. */
dg_status dg_use_graphs(dg_ctx* ctx, int enable);

/* Per-kernel timing (instrumentation for measurement): while enabled, every
 * launch of the listed kernel families on the context's stream is bracketed
 * by HIP events.  dg_timing(ctx, 1) enables and clears, dg_timing(ctx, 0)
 * disables.  dg_timing_read synchronises the stream and returns, per family,
 * the summed device time (ms), the launch count and the summed algorithmic
 * bytes and flops of those launches (what the operation must move/compute:
 * residual 16 B/DOF, FD J.v 32 B/DOF, exact J.v 24 B/DOF, diagonal blocks the
 * written blocks, PLU (2/3) n^3 flops and one read + write of the block,
 * block-Jacobi apply one read of the factors (or inverse) and 16 B per vector
 * entry, block-sparse coarse product its 7 blocks per element and 16 B per
 * entry, Arnoldi step j 24 (j + 1) + 32 B per entry: the dots, the first
 * update with the second-pass dots and the norm, the second update with the
 * normalisation; 16 (j + 1) + 32 when the first dots are taken inside the
 * coarse product) since the last clear, then clears.  The fine-level (level 0)
 * block-Jacobi apply is its own family; coarse-level applies form another.
 * All arrays have DG_K_COUNT entries (host memory). */
enum { DG_K_RESIDUAL = 0, DG_K_JVP_FD = 1, DG_K_JVP_EXACT = 2, DG_K_DIAG_BLOCKS = 3, DG_K_LU = 4,
       DG_K_BJ_FINE = 5, DG_K_BSR = 6, DG_K_BJ_COARSE = 7, DG_K_ARNOLDI = 8, DG_K_COUNT = 9 };
dg_status dg_timing(dg_ctx* ctx, int enable);
dg_status dg_timing_read(dg_ctx* ctx, double* ms, int* counts, double* bytes, double* flops);


/* ---- Batches of independent cases -------------------------------------------
 * A batch holds many independent cases (each its own periodic mesh, gas and
 * degree p), one context per case on its own stream.  Batched vectors are the
 * concatenation of the cases' vectors in case order: case c occupies
 * dg_batch_ndof(b, c) entries from dg_batch_offset(b, c), each in the layout of
 * a single context.  The DG operator of all cases (residual Sec. 3.1 Eq. re;
 * FD product Sec. 5.1 Eq. DG-mf with a per-case step h_c computed from the
 * case's own norms; exact product) runs as ONE persistent launch over a device
 * work list of (case, element tile) items, each taking the compiled path of
 * its degree; results equal the single-context calls bitwise.  Every case of a
 * batch must share Euler/Navier-Stokes and straight/curved.  Calls enqueue on
 * the batch stream hip_stream (NULL = the default stream); graphs are
 * captured on a private stream and launched on the batch stream. */
typedef struct dg_batch dg_batch;

typedef struct {
    dg_mesh_desc mesh;
    dg_phys phys;
    int p;
} dg_case_desc;

/* Tile shape of one batched kernel kind: workgroup size, elements per
 * workgroup for each degree (epb[1..4]; 0 = degree absent), persistent grid,
 * dynamic LDS bytes, measured ms per launch (-1 if not tuned), candidates
 * timed by the autotuner and work items. */
typedef struct {
    int threads;
    int epb[5];
    int grid;
    size_t lds_bytes;
    double ms;
    int candidates;
    int items;
} dg_batch_tile;

dg_status dg_batch_create(const dg_case_desc* cases, int ncases, void* hip_stream, dg_batch** out);
dg_status dg_batch_destroy(dg_batch* b);
const char* dg_batch_last_error(const dg_batch* b);
/* Entries of case c (c < 0: the whole batch) and its first entry. */
size_t dg_batch_ndof(const dg_batch* b, int c);
size_t dg_batch_offset(const dg_batch* b, int c);
/* The context of case c (owned by the batch; valid until dg_batch_destroy):
 * every single-context entry point can be used on it, on the case's stream. */
dg_ctx* dg_batch_case(dg_batch* b, int c);
/* R = R(W) for every case (Sec. 3.1 Eq. re). */
dg_status dg_batch_residual(dg_batch* b, const double* W, double* R);
/* y_c = shift M v_c + (R(W_c + h_c v_c) - RW_c) / h_c,
 * h_c = 1e-7 sqrt(1 + ||W_c||) / ||v_c|| (Sec. 5.1 Eq. DG-mf).  Replayed as a
 * HIP graph when called again with the same pointers and shift. */
dg_status dg_batch_jvp(dg_batch* b, const double* W, const double* RW, const double* v, double shift, double* y);
/* y_c = shift M v_c + J(W_c) v_c exactly (tangent-linear). */
dg_status dg_batch_jvp_exact(dg_batch* b, const double* W, const double* v, double shift, double* y);
dg_status dg_batch_use_graphs(dg_batch* b, int enable);
/* kind: DG_K_RESIDUAL, DG_K_JVP_FD or DG_K_JVP_EXACT. */
dg_status dg_batch_get_tile(dg_batch* b, int kind, dg_batch_tile* t);
/* Fix a tile shape: threads 64..256 (multiple of 64), LDS cap in bytes (a
 * degree whose element slot needs more still gets one element), persistent
 * grid of grid_per_cu workgroups per CU (at most the number of items). */
dg_status dg_batch_set_tile(dg_batch* b, int kind, int threads, size_t lds_cap, int grid_per_cu);
/* Autotuner: time every candidate shape (threads 64/128/192/256, LDS caps
 * 32/64/96/160 KB, 1/2/4/8 workgroups per CU) on the given operands, `reps`
 * launches each, and keep the fastest for this kind (chosen may be NULL).
 * RW is needed for DG_K_JVP_FD, v for both products.  Synchronises. */
dg_status dg_batch_tune(dg_batch* b, int kind, const double* W, const double* RW, const double* v, int reps,
                        dg_batch_tile* chosen);
/* One BDF2 step (as dg_bdf2_step) of every case: popts[c] is case c's
 * preconditioner, fopts/newton_rtol/max_newton are shared, stats[c] (may be
 * NULL) receives case c's statistics.  `workers` host threads run the cases,
 * largest first, each on its own stream.  Synchronous.  Returns DG_ENOCONV
 * (all steps completed) if some case missed its tolerance. */
dg_status dg_batch_bdf2_step(dg_batch* b, const double* Wn, const double* Wnm1, double dt, const pmg_opts* popts,
                             const fgmres_opts* fopts, double newton_rtol, int max_newton, int workers, double* Wnp1,
                             dg_step_stats* stats);

/* ---- Device memory ------------------------------------------------------------
 * dg_device_bytes: device memory the context holds now.
 * dg_footprint_bytes: what a context of this mesh and degree allocates for one
 * BDF2 step with these options (create, pmg_setup, FGMRES Krylov basis,
 * Newton vectors, graph staging): factors, coarse operators and Krylov bases
 * dominate.  Host-only arithmetic, no GPU needed; -1 on bad arguments. */
double dg_device_bytes(const dg_ctx* ctx);
double dg_footprint_bytes(const dg_mesh_desc* mesh, int p, const pmg_opts* popts, const fgmres_opts* fopts);

/* ---- Serving loop -----------------------------------------------------------------
 * Requests are implicit time steps (one dg_bdf2_step each) on straight periodic
 * boxes.  `slots` worker threads each run one request at a time on the
 * request's own stream, so up to `slots` requests overlap on the GPU.
 * Admission is first-in first-out: the oldest waiting request starts when a
 * slot is free and its footprint (dg_footprint_bytes) fits in hbm_budget next
 * to the contexts the server holds (idle cached contexts are freed, least
 * recently used first, to make room); a request that can never fit completes
 * with DG_ENOMEM.  With cache = 1 a finished request's context stays resident
 * and serves later requests of the same mesh, degree, gas and solver options.  Results do not
 * depend on what else runs: each request's arithmetic is that of dg_bdf2_step
 * on its own context.  Wn, Wnm1 (may be NULL) and Wnp1 are caller-owned
 * device vectors: the inputs must be written (their producing work complete)
 * before dg_server_submit, since the step runs on a stream of its own, and all
 * three must stay valid until the request's response is polled; Wnp1 is
 * complete when its response is returned.  Times are seconds on the server's
 * clock (dg_server_time). */
typedef struct dg_server dg_server;

typedef struct {
    int slots;              /* concurrent requests, 1..64                         */
    double hbm_budget;      /* bytes of contexts the server may hold (0: 85% of
                               the free device memory at creation)              */
    int cache;              /* keep idle contexts for reuse (1) or free them (0) */
} dg_server_opts;

typedef struct {
    dg_mesh_desc mesh;      /* vtx must be NULL                                   */
    dg_phys phys;
    int p;
    double dt;
    pmg_opts popts;
    fgmres_opts fopts;
    double newton_rtol;
    int max_newton;
    const double* Wn;
    const double* Wnm1;
    double* Wnp1;
    long long tag;          /* returned in the response                           */
} dg_request;

typedef struct {
    long long tag;
    int status;             /* dg_status of the step                              */
    int concurrent;         /* requests running when this one was admitted       */
    double t_submit, t_admit, t_done;
    double footprint;       /* bytes charged at admission                         */
    double device_bytes;    /* bytes the context held after the step             */
    size_t ndof;
    dg_step_stats stats;
} dg_response;

typedef struct {
    long long submitted, completed, pending;
    int running, contexts;
    double held_bytes, peak_held_bytes, budget_bytes;
} dg_server_info;

dg_status dg_server_create(const dg_server_opts* opts, dg_server** out);
dg_status dg_server_destroy(dg_server* sv);   /* finishes queued requests first  */
const char* dg_server_last_error(const dg_server* sv);
double dg_server_time(const dg_server* sv);
/* Queue one request (copied); returns at once. */
dg_status dg_server_submit(dg_server* sv, const dg_request* rq);
/* Move up to max finished responses to out (oldest first), waiting up to
 * wait_ms for one if none is ready; returns the count (-1 on bad arguments). */
int dg_server_poll(dg_server* sv, dg_response* out, int max, int wait_ms);
/* Wait until every submitted request has finished. */
dg_status dg_server_drain(dg_server* sv);
dg_status dg_server_stats(dg_server* sv, dg_server_info* info);

#ifdef __cplusplus
}
#endif
#endif
