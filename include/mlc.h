/*
 * mlc.h -- C ABI of the MI355X (gfx950) library for the multilevel local-and-parallel
 * finite element eigen-correction of Li, Han, Xie and You (arXiv:1401.4969).
 *
 * Problem (Section 3, eigenproblem (Weak_Eigenvalue_Problem) with the operator of
 * Section 2.2, A = kappa I): find (lambda, u) with -div(kappa grad u) = lambda u in Omega,
 * u = 0 on the boundary, b(u, u) = 1 -- or, with MLC_COEF_TENSOR, the operator of
 * Example 6.2: -div(A grad u) = lambda phi u, A a full symmetric tensor and phi > 0 a
 * weight, b(u, v) = (phi u, v) -- discretised by conforming P1 or P2 elements (Section
 * 2.1) on nested uniform right-triangle meshes (each square cell cut by its lower-left to
 * upper-right diagonal; regular refinement, beta = 2, Section 6).
 *
 * Method (Algorithm 4.2 driving Algorithm 4.1):
 *   mlc_coarse_setup    -- Algorithm 4.2 step 1: the eigenproblem on the coarse space
 *                          V_0H (h_1 = H), solved once; its eigenbasis is kept for step 3.
 *   mlc_level_correct   -- one Correction(V_0H, lambda_hk, u_hk, V_0h_{k+1}) of
 *                          Algorithm 4.1: (1) independent local solves of equation
 *                          (Aux_Problem) on every overlapping subdomain Omega_j,
 *                          (2) partition-of-unity gluing of the corrections into u~,
 *                          (3) Rayleigh-Ritz (Eigen_Augment_Problem) on V_0H + span{u~}.
 *   mlc_get_eigenpairs  -- the current (lambda, u), b(u_i, u_j) = delta_ij.
 *
 * Conventions
 *   - Every call returns an mlc_status; no C++ exception or abort crosses the ABI.
 *   - Device buffers are plain device pointers (hipMalloc'd or any device allocation).
 *     The caller owns all device memory: the workspace passed to mlc_create and every
 *     output buffer.  The library allocates no device memory of its own except the
 *     internal buffers of the dense generalized eigensolver used once by
 *     mlc_coarse_setup (rocSOLVER).
 *   - All work is enqueued on the caller's HIP stream (borrowed, never destroyed) and is
 *     stream-ordered; only calls that return host data synchronise that stream.
 *   - Grid vectors are full node grids of the bounding box, row-major: the value at node
 *     (i, j) (x = x0 + i h, y = y0 + j h) is at index j*(N+1)+i, N = n_coarse*2^level
 *     cells per side (P1); with P2 elements the grid has 2N intervals of h/2 (vertices and
 *     edge midpoints); boundary and removed-quadrant nodes hold 0.  q eigenvectors are
 *     stored one after another.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef MLC_H
#define MLC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mlc_status {
  MLC_OK = 0,
  MLC_EINVAL = 1,   /* invalid argument or unsupported problem */
  MLC_ENOMEM = 2,   /* workspace too small */
  MLC_EHIP = 3,     /* a HIP runtime or library call failed; see mlc_last_error */
  MLC_ENOCONV = 4,  /* a local solve (or, with MLC_POU_INTERFACE, the G_{m+1} problem) did
                       not reach its tolerance within max_it; results are still written.
                       Reported by mlc_level_correct with statistics, mlc_run,
                       mlc_batch_step_stats and mlc_batch_run */
  MLC_ESTATE = 5    /* call out of order (e.g. level_correct before coarse_setup) */
} mlc_status;

enum { MLC_DOMAIN_SQUARE = 0,   /* (0,1)^2 */
       MLC_DOMAIN_LSHAPE = 1,   /* (-1,1)^2 \ [0,1)x(-1,0] */
       MLC_DOMAIN_SQUARE2 = 2 };/* (-1,1)^2 (Example 6.2) */

enum { MLC_COEF_ONE = 0,        /* kappa == 1 */
       MLC_COEF_COARSE = 1,     /* one kappa per coarse cell, [n_coarse*n_coarse] */
       MLC_COEF_FINE = 2,       /* one kappa per finest square cell, [N_L*N_L] */
       MLC_COEF_TENSOR = 3 };   /* Example 6.2: per finest triangle a symmetric positive definite
                                   A and a mass weight phi > 0, [4][2][N_L][N_L]: component
                                   (a11, a12, a22, phi), triangle (0 below the SW-NE diagonal,
                                   1 above), row J along y, column I along x.  Each value is
                                   taken constant on its triangle and every level integrates
                                   the forms exactly (seven-point stencils, Galerkin coarse
                                   levels).  Not available with record_tape. */

/* Gluing of the local corrections, u~ = I u + sum_j chi_j e^j with chi_j = phi_j / sum_l phi_l
   (a partition of unity in place of the G_j / G_{m+1} construction of Algorithm 4.1 step 2): */
enum { MLC_POU_RAMP = 0,        /* phi_j = rho(x) rho(y): 1 on D_j, linear to 0 across the overlap */
       MLC_POU_INDICATOR = 1,   /* phi_j = indicator of the closed D_j (allows overlap 0) */
       MLC_POU_INTERFACE = 2 }; /* not a partition of unity: Algorithm 4.1 step 2 as stated,
                                   u~ = u~^j on G_j = D_j shrunk by half a coarse cell, and on
                                   G_{m+1} (the rest) the Dirichlet problem of equation
                                   (G_m+1_Problem), solved by a global CG; single-problem
                                   contexts without a tape only */

enum { MLC_PREC_FP64 = 0,       /* every local solve in FP64 */
       MLC_PREC_MIXED = 1 };    /* FP32 inner PCG with FP64 residual refinement */

/* Problem description (Section 3 eigenproblem; Section 4 domain decomposition). */
typedef struct mlc_problem_desc {
  int32_t domain;      /* MLC_DOMAIN_* */
  int32_t n_coarse;    /* coarse cells per bounding-box side; H = side/n_coarse (even for the L-shape) */
  int32_t n_refine;    /* number of corrections L; finest h = H/2^L; level 0 is the coarse mesh */
  int32_t sub_x;       /* D_j blocks along x: boundaries at floor(b*n_coarse/sub_x) coarse cells */
  int32_t sub_y;       /* D_j blocks along y */
  int32_t overlap;     /* Omega_j = D_j grown by this many coarse cells per side (>= 1 with
                          MLC_POU_RAMP, >= 0 otherwise); every Omega_j must be at least 2
                          coarse cells wide and tall */
  int32_t n_eig;       /* q, number of lowest eigenpairs (1..8) */
  int32_t coef_kind;   /* MLC_COEF_*; for kinds 1 and 2 both triangles of a square cell
                          share its value */
  const double* kappa; /* host pointer, row-major [row along y][col along x] (kind 3: the
                          layout of MLC_COEF_TENSOR); read during mlc_create only (copied);
                          NULL for MLC_COEF_ONE.  Must be > 0 and finite. */
  int32_t pou;         /* MLC_POU_* (0 unless set) */
  int32_t order;       /* element degree: 1 (P1, also 0) or 2 (P2: values at the vertices and
                          edge midpoints, i.e. the nodes of the grid with twice the cells'
                          intervals; coef_kind 0 or 1, pou 0 or 1, FP64, no tape).  Grid
                          vectors of level l then have n_coarse*2^(l+1)+1 nodes per side. */
} mlc_problem_desc;

/* Solver options; mlc_default_opts fills the defaults shown. */
typedef struct mlc_solver_opts {
  int32_t precision;   /* MLC_PREC_FP64 (default) or MLC_PREC_MIXED */
  double rtol;         /* local solve: ||r||_2 <= rtol * ||b||_2 from a zero guess (1e-12) */
  int32_t max_it;      /* PCG iterations per local solve (FP64) or per inner solve (200) */
  int32_t max_refine;  /* mixed precision: FP64 refinement steps (10) */
  double inner_rtol;   /* mixed precision: FP32 inner solve relative tolerance (1e-4) */
  int32_t nu;          /* damped Jacobi sweeps before and after each coarse correction (2) */
  double omega;        /* Jacobi damping (0.8) of every sweep with smoother 0, or with nu != 2 */
  int32_t block;       /* threads per workgroup of the local solver: 256, 512 or 1024 (0 = 1024) */
  int32_t timing;      /* 1: record HIP events around the local-solve kernel (see mlc_phase_times) */
  int32_t record_tape; /* 1: keep every level's forward state for mlc_backward (single problem,
                          q = 1, coef_kind 1 or 2; enlarges the workspace) */
  int32_t glue_graph_it; /* MLC_POU_INTERFACE in hipGraph batch steps: CG iterations of the
                          G_{m+1} problem in the captured sequence (24; 1..1000); right-hand
                          sides that converge earlier are frozen, and one that has not
                          converged by then makes the step's statistics and mlc_batch_run
                          report MLC_ENOCONV.  Eager steps iterate to convergence (at most
                          1000 iterations). */
  int32_t smoother;    /* sweeps of the local solves' V-cycle with nu = 2: 1 (default) the two
                          damping factors of the degree-2 Chebyshev polynomial of [1/2, 2]
                          (1.3895, 0.5617; the part of the spectrum of D^-1 K that the coarse
                          grid leaves), 0 damped Jacobi with omega for both */
} mlc_solver_opts;

/* Per-level statistics, filled by mlc_level_correct when st != NULL (this synchronises
 * the stream). */
typedef struct mlc_level_stats {
  int32_t level;        /* level produced (k+1) */
  int32_t n_items;      /* local solves launched (kept subdomains x q) */
  double h;             /* mesh size of that level */
  int64_t n_dofs;       /* interior nodes of the level */
  int64_t n_tile_dofs;  /* sum over local solves of their unknowns */
  int32_t it_max;       /* max PCG iterations over the local solves (inner, for mixed) */
  int32_t refine_max;   /* mixed precision: max FP64 refinement steps */
  int64_t it_sum;       /* sum of PCG iterations over the local solves */
  int64_t it_dofs;      /* sum over local solves of iterations x unknowns */
  double relres_max;    /* max final ||r||/||b|| over the local solves */
  double lambda[8];     /* the q eigenvalues after the step */
  int64_t refine_dofs;  /* mixed precision: sum over local solves of refinement steps x unknowns */
  int32_t glue_it;      /* MLC_POU_INTERFACE: CG iterations of the G_{m+1} problem (max over rhs) */
  double glue_relres;   /* MLC_POU_INTERFACE: its final ||r||/||r_0|| (max over rhs) */
} mlc_level_stats;

/* Fill opts with the defaults listed above. */
mlc_status mlc_default_opts(mlc_solver_opts* opts);

/* Bytes of device workspace mlc_create needs for this problem and these options. */
mlc_status mlc_workspace_size(const mlc_problem_desc* desc, const mlc_solver_opts* opts,
                              size_t* bytes);

/* Create a context.  dev_workspace: device buffer of at least mlc_workspace_size bytes,
 * 256-byte aligned, owned by the caller and kept alive until mlc_destroy.  hip_stream:
 * a hipStream_t (NULL = default stream).  Uploads geometry tables on the stream.
 * MLC_EINVAL (mlc_workspace_size and the batch calls reject the same) for:
 *   descriptor: NULL; domain outside 0..2; coef_kind outside 0..3; n_coarse outside
 *   2..4096, or odd on the L-shape; n_refine outside 1..10; a finest grid of more than
 *   32768 cells per side (n_coarse * 2^n_refine); sub_x or sub_y outside 1..n_coarse; pou
 *   outside 0..2; overlap above n_coarse, or below 1 with MLC_POU_RAMP (below 0
 *   otherwise); an Omega_j narrower than 2 coarse cells either way; more than 8 blocks
 *   D_j whose Omega_j reach one node along an axis (overlap too wide for the blocks);
 *   a subdomain whose coarse interior exceeds 1024 nodes; n_eig outside 1..8 or above the
 *   number of coarse interior nodes n_H; n_H (1 + 4 n_eig) + n_eig^2 above 18432 (the
 *   LDS of the device Rayleigh-Ritz solve, 144 KiB); kappa NULL when the kind needs it, or a value not > 0 and
 *   finite (kind 3: A not positive definite or phi not > 0 on some triangle);
 *   MLC_POU_INTERFACE with a tape or in a batch of more than one problem; record_tape
 *   with n_eig != 1 or coef_kind other than 1 and 2; order other than 0, 1 and 2; order 2
 *   with coef_kind 2 or 3, MLC_POU_INTERFACE, mixed precision or a tape, or a finest node
 *   grid above 32768 intervals per side; problems of one batch with different order;
 *   options: NULL; precision not 0 or 1; rtol outside (0, 1); max_it < 1; nu outside
 *   1..8; omega outside (0, 1); mixed precision with max_refine < 1 or inner_rtol outside
 *   (0, 1); block not 0, 256, 512 or 1024; glue_graph_it outside 1..1000; smoother not 0
 *   or 1;
 *   workspace: NULL or not 256-byte aligned (MLC_ENOMEM when smaller than needed). */
mlc_status mlc_create(const mlc_problem_desc* desc, const mlc_solver_opts* opts,
                      void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                      struct mlc_ctx** out);

/* Algorithm 4.2 step 1 with h_1 = H: coefficients on every level (children means),
 * coarse stiffness and mass, the full generalized eigendecomposition on V_0H, the
 * initial eigenpairs (level 0), and the exact coarsest-grid inverses of every
 * subdomain.  Synchronises the stream. */
mlc_status mlc_coarse_setup(struct mlc_ctx* ctx);

/* One correction step (Algorithm 4.1) from the current level k to k+1.  Stream-ordered
 * and asynchronous when st == NULL.  MLC_ESTATE before setup or at the finest level. */
mlc_status mlc_level_correct(struct mlc_ctx* ctx, mlc_level_stats* st);

/* Run every remaining correction (no statistics); then synchronise and return
 * MLC_ENOCONV if a local solve of any of these steps ended above rtol (mlc_level_correct
 * without statistics is asynchronous and reports nothing). */
mlc_status mlc_run(struct mlc_ctx* ctx);

/* Step back to the previous level (its eigenpair is still held), so the last
 * correction can be repeated.  MLC_ESTATE if there is none. */
mlc_status mlc_rewind(struct mlc_ctx* ctx);

/* Current level k (0 after setup, L at the end). */
mlc_status mlc_current_level(const struct mlc_ctx* ctx, int32_t* level);

/* The current eigenpairs: lambda_host[q] (host, may be NULL) and u_dev (device,
 * q*(N_k+1)^2 doubles, may be NULL).  b(u, u) = 1 leaves the sign free; each eigenvector
 * is signed so that its nodal sum is positive when |sum u| > 1e-8 sum |u|, and otherwise
 * (a vector odd under a symmetry of the problem) so that the first node in grid order
 * whose magnitude is within a relative 1e-6 of the largest is positive.  Synchronises
 * the stream when lambda_host != NULL. */
mlc_status mlc_get_eigenpairs(struct mlc_ctx* ctx, double* lambda_host, double* u_dev);

/* Replace the current state by (level, lambda_host[q], u_dev) given on the level grid
 * (device, q*(N_level+1)^2 doubles, values at non-interior nodes ignored).  Needs setup.
 * The recorded tape of the levels up to `level` then no longer belongs to the state:
 * mlc_backward and mlc_hf_gradient return MLC_ESTATE until the next mlc_coarse_setup and
 * a run from level 0. */
mlc_status mlc_set_state(struct mlc_ctx* ctx, int32_t level, const double* lambda_host,
                         const double* u_dev);

/* Accumulated milliseconds measured with HIP events on the stream since the last call:
 * ms[0] = local-solve kernel, ms[1] = whole level_correct calls.  Synchronises. */
mlc_status mlc_phase_times(struct mlc_ctx* ctx, double* ms, int32_t n);

/* Exact reverse-mode derivative of the computed finest eigenvalue lambda_1 with respect to
 * the coefficient, through every level: the coarse eigenproblem (Algorithm 4.2 step 1),
 * every correction step (local solves, gluing, Rayleigh-Ritz of Algorithm 4.1) and the
 * children-mean coefficients of coarser levels.  lambda_bar_host (host, one double, read)
 * is the incoming adjoint of lambda_1; kappa_bar_dev (device, written) receives
 * lambda_bar * d lambda_1 / d kappa in the layout of desc->kappa: per finest cell
 * (coef_kind 2) or per coarse cell (coef_kind 1).  MLC_EINVAL for a NULL pointer or
 * without opts.record_tape = 1; MLC_ESTATE without a complete forward run from level 0
 * (coarse_setup, then every level_correct; not after mlc_set_state).  Runs one adjoint
 * local solve per subdomain and level.  Synchronises. */
mlc_status mlc_backward(struct mlc_ctx* ctx, const double* lambda_bar_host, double* kappa_bar_dev);

/* Hellmann-Feynman reference gradient: (u, dK/dkappa u) for the finest eigenvector
 * (b(u,u) = 1), same layout and requirements as mlc_backward.  It ignores how the
 * multilevel approximation itself depends on kappa, so it differs from mlc_backward by
 * the approximation error; it is a reference, not the derivative. */
mlc_status mlc_hf_gradient(struct mlc_ctx* ctx, double* kappa_bar_dev);

mlc_status mlc_destroy(struct mlc_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the whole of Algorithm 4.2 in one call --
 * mlc_create, mlc_coarse_setup, mlc_run, mlc_get_eigenpairs and mlc_destroy -- with the
 * library's static device scratch array (64 MiB per device, held until the process ends) as
 * the workspace instead of a caller's buffer.  Calls no hipMalloc, hipFree or allocating
 * library routine: the coarse eigendecomposition runs on the device, so the problem's
 * coarse space may have at most 400 nodes (MLC_EINVAL above that, and with record_tape or
 * timing set); MLC_ENOMEM when mlc_workspace_size exceeds 64 MiB.  lambda_host (host, q
 * doubles) and u_dev (device, q*(N_L+1)^2 doubles, may be NULL) as in mlc_get_eigenpairs;
 * MLC_ENOCONV as mlc_run (results written).  Synchronises the stream.  Every call on one
 * device shares that device's scratch array and leaves its contents behind: calls that
 * overlap on one device (other threads, other streams) race. */
mlc_status mlc_solve_static(const mlc_problem_desc* desc, const mlc_solver_opts* opts,
                            void* hip_stream, double* lambda_host, double* u_dev);

/* ---- Batches: many independent problems, one launch per kernel and level step ----
 *
 * All problems of a batch share q (n_eig) and coef_kind; domains, meshes, subdomain
 * grids, coefficients and numbers of levels may differ.  Step s produces level s of every
 * problem with n_refine >= s; the local solves of all those problems (of uneven sizes)
 * run in one launch, ordered largest tile first.  Same conventions as above: caller-owned
 * workspace, borrowed stream, statuses. */
typedef struct mlc_batch mlc_batch;

/* Workspace bytes for n problems (descs[0..n-1]); MLC_EINVAL as for mlc_create, or for
 * n < 1 or mixed q / coef_kind. */
mlc_status mlc_batch_workspace_size(int32_t n, const mlc_problem_desc* descs,
                                    const mlc_solver_opts* opts, size_t* bytes);

/* Create a batch context over a caller-owned device workspace (256-byte aligned). */
mlc_status mlc_batch_create(int32_t n, const mlc_problem_desc* descs, const mlc_solver_opts* opts,
                            void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                            mlc_batch** out);

/* Algorithm 4.2 step 1 for every problem (as mlc_coarse_setup).  Synchronises. */
mlc_status mlc_batch_setup(mlc_batch* b);

/* One level step for every problem that has it.  use_graph = 1 captures the step's
 * launch sequence in a hipGraph on first use and replays it afterwards.  MLC_ESTATE
 * before setup or after the last step. */
mlc_status mlc_batch_step(mlc_batch* b, int32_t use_graph);

/* All remaining steps (Algorithm 4.2 for every problem); then synchronise and return
 * MLC_ENOCONV if a local solve of any of these steps ended above rtol. */
mlc_status mlc_batch_run(mlc_batch* b, int32_t use_graph);

/* Step back once (the previous eigenpairs are still held), so a step can be repeated. */
mlc_status mlc_batch_rewind(mlc_batch* b);

/* Back to step 0 (the level-0 eigenpairs from the stored coarse eigenbasis) without
 * redoing the setup, e.g. to time repeated full runs.  Stream-ordered. */
mlc_status mlc_batch_restart(mlc_batch* b);

/* Current step (0 after setup). */
mlc_status mlc_batch_current_step(const mlc_batch* b, int32_t* step);

/* Eigenpairs of problem i at its current level (min(step, n_refine_i)): lambda_host[q]
 * (host, may be NULL), u_dev (device, q*(N+1)^2, may be NULL), signed as in
 * mlc_get_eigenpairs.  Synchronises when lambda_host != NULL. */
mlc_status mlc_batch_get(mlc_batch* b, int32_t i, double* lambda_host, double* u_dev);

/* Statistics of the last step aggregated over the batch (synchronises): st->level is the
 * step, n_dofs the interior nodes of all problems at that step, lambda[] unused. */
mlc_status mlc_batch_step_stats(mlc_batch* b, mlc_level_stats* st);

/* Autotuner: per step, the workgroup size of the local solves (256, 512 or 1024 threads),
 * nu (1..3) and, with mixed precision, the inner FP32 tolerance (1e-3, 3e-4, 1e-4, 3e-5,
 * 1e-5), by a
 * coordinate search: the sizes at the batch's nu and tolerance, then nu at the chosen
 * sizes, then the tolerance.  Each candidate is timed over three full runs from level 0
 * (HIP events around the local-solve launches, the median per step); every setting
 * solves to the same rtol, so the choice changes only the time (and rounding).
 * blocks_out (may be NULL) receives the sizes per step (index s-1, n entries); see
 * mlc_batch_get_tuning for the rest.  The choice is cached in a text file
 * (MLC_AUTOTUNE_CACHE, else $HOME/.cache/mlc_autotune.txt; one line per key, "block nu
 * inner_rtol" per step) under a key of the device architecture and a hash of what decides
 * the launches (element order, coefficient kind, precision, q, the created nu and inner
 * tolerance, every item's subdomain shape); a later call with the same key, in any
 * process, takes the cached choice without timing.  Leaves the batch at step 0.
 * Synchronises. */
mlc_status mlc_batch_autotune(mlc_batch* b, int32_t* blocks_out, int32_t n);

/* Use these workgroup sizes per step (index s-1; 256, 512 or 1024), e.g. a cached
 * autotuner result.  Drops captured graphs. */
mlc_status mlc_batch_set_blocks(mlc_batch* b, const int32_t* blocks, int32_t n);

/* The per-step settings of the local solves (index s-1, up to n steps; any output may be
 * NULL): workgroup size, nu, inner FP32 tolerance (used with mixed precision). */
mlc_status mlc_batch_get_tuning(const mlc_batch* b, int32_t* blocks, int32_t* nu,
                                double* inner_rtol, int32_t n);

/* Set them (e.g. an autotuner result of another batch): MLC_EINVAL unless every step has
 * block 256, 512 or 1024, nu in 1..8 and inner_rtol in (0, 1).  Drops captured graphs. */
mlc_status mlc_batch_set_tuning(mlc_batch* b, const int32_t* blocks, const int32_t* nu,
                                const double* inner_rtol, int32_t n);

/* As mlc_phase_times, for steps run without graphs. */
mlc_status mlc_batch_phase_times(mlc_batch* b, double* ms, int32_t n);

mlc_status mlc_batch_destroy(mlc_batch* b);
const char* mlc_batch_last_error(const mlc_batch* b);


const char* mlc_status_str(mlc_status s);
/* Message of the last failure on this context (never NULL; "" if none). */
const char* mlc_last_error(const struct mlc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MLC_H */
