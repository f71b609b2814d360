/*
 * stwr.h - C ABI of the space-time waveform-relaxation multigrid library for
 * incompressible Navier-Stokes on one AMD Instinct MI355X (gfx950).
 *
 * Method: Taylor-Hood P2-P1 (or P3-P2, degree = 2) in space times upwind DG(q)
 * in time (q in {0,1}),
 * solved all at once in space-time by Newton's method, FGMRES preconditioned
 * by geometric multigrid V-cycles whose smoother is the waveform-relaxation
 * Vanka+star patch relaxation with Chebyshev weights.  Paper sections:
 *   weak form ............. Sec. 2, eq. nsfem (with eq. dgintime)
 *   V-cycle ............... Sec. 3, Alg. 1
 *   FGMRES, Chebyshev ..... Sec. 3 (interval [0.25 lam, 1.05 lam], 10-step estimate)
 *   transfers ............. Sec. 3, P = I (x) blockdiag(P_u, P_phi), R = P^T
 *   patch relaxation ...... Sec. 3 Vanka+star patches, eq. waveform_patch_solve
 *   Newton ................ Sec. 4.2
 *   heat equation ......... Sec. 2, eq. heatfem; vertex-star patches, Sec. 3;
 *                           FGMRES-WRMG runs of Sec. 4.1 (equation = STWR_EQ_HEAT)
 *
 * Conventions shared by every call
 * ---------------------------------
 * Mesh: unit square, mesh_n x mesh_n squares, each cut from bottom-right to
 *   top-left.  Level 0 is the finest; level l has mesh_n >> l squares a side.
 * Free spatial DoFs of a level with M squares a side (Dirichlet velocity DoFs
 *   on the boundary are eliminated): interior P2 node k = (gi-1) + (2M-1)(gj-1)
 *   (gi, gj in 1..2M-1 on the (2M+1)^2 node grid of spacing 1/(2M)) owns
 *   velocity DoFs 2k (x) and 2k+1 (y); the pressure at vertex v = i + (M+1) j
 *   is DoF 2(2M-1)^2 + v.
 * Space-time vectors: float64, length n_st = n_free * n_slabs * (q+1), index
 *   (dof * n_slabs + n) * (q+1) + a, i.e. [free DoF][slab][temporal node];
 *   the temporal nodes of each slab are the family the problem descriptor's
 *   temporal_nodes names (right Gauss-Radau by default, or Gauss-Legendre).
 * Memory: every vector argument is a DEVICE pointer on the context's device,
 *   owned by the caller, non-overlapping unless stated.  Work is enqueued on
 *   the context's stream; calls that return host scalars synchronise it.
 * Errors: every call returns an stwr_status; no C++ exception crosses the
 *   ABI.  stwr_last_error() gives the message of the last failure on the
 *   context.  On STWR_ERR_ARG and STWR_ERR_BUDGET outputs are untouched.
 */
#ifndef STWR_H
#define STWR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STWR_OK = 0,
  STWR_ERR_ARG = -1,           /* bad argument (null pointer, level out of range, ...) */
  STWR_ERR_OOM = -2,           /* device allocation failed */
  STWR_ERR_BUDGET = -3,        /* problem does not fit the context's HBM budget */
  STWR_ERR_DEVICE = -4,        /* HIP runtime error */
  STWR_ERR_SINGULAR = -5,      /* a patch or coarse block had a zero/non-finite pivot */
  STWR_ERR_NONFINITE = -6,     /* NaN/Inf met in a residual norm */
  STWR_ERR_NOT_CONVERGED = -7, /* iteration limit reached (stats still filled) */
  STWR_ERR_STATE = -8          /* call made before the data it needs exists */
} stwr_status;

enum { STWR_FP64 = 0, STWR_FP32 = 1 };

typedef struct stwr_ctx stwr_ctx;
typedef struct stwr_problem stwr_problem;

/* One space-time Navier-Stokes problem (manufactured solution, Sec. 2 forms
 * with forcing).  The modes are read during stwr_problem_create and copied:
 *   psi(t,x,y) = sum_m c_m sin(a_m pi x) sin(b_m pi y) cos(w_m t + th_m),
 *   u = (d psi/dy, -d psi/dx),
 *   p(t,x,y)   = sum_m d_m cos(al_m pi x) cos(be_m pi y) cos(w'_m t + th'_m).
 * psi_ab: host int32[n_psi_modes][2] = (a, b); psi_coef: host f64[n][3] =
 * (c, w, th); p_ab: host int32[n_p_modes][2]; p_coef: host f64[n][3].
 * mesh_n must be divisible by 2^(n_levels-1) with mesh_n >> (n_levels-1) >= 2;
 * q in {0, 1}; n_slabs >= 1. */
typedef struct {
  int32_t mesh_n, n_levels, q, n_slabs;
  double t_final, reynolds;
  int32_t n_psi_modes, n_p_modes;
  const int32_t* psi_ab;
  const double* psi_coef;
  const int32_t* p_ab;
  const double* p_coef;
  int32_t flow;   /* STWR_FLOW_MODES: the modes above; STWR_FLOW_CHORIN, STWR_FLOW_CAVITY: below */
  int32_t temporal_nodes;  /* STWR_NODES_RADAU (default) or STWR_NODES_GAUSS, see below */
  int32_t equation;        /* STWR_EQ_NAVIER_STOKES (default) or STWR_EQ_HEAT, see below */
  int32_t degree;          /* heat: spatial degree k of P_k, 1..3; Navier-Stokes: pressure degree k
                              of Taylor-Hood P_{k+1}-P_k, 2 for P3-P2 (Sec. 3.1), 0 or 1 for P2-P1 */
} stwr_problem_desc;

/* equation = STWR_EQ_HEAT selects the heat equation u_t - Laplace u = 0 of
 * Sec. 2 (eq. heatfem) on the unit square with natural (homogeneous Neumann)
 * boundary conditions, scalar continuous P_k in space (k = degree, 1..3) and
 * DG(q) in time (q in 0..3), initial value the nodal interpolant of
 * u_0 = sin(pi x) + cos(2 pi y) (the paper's runs, Sec. 4.1).  Reynolds
 * number, modes and flow are ignored.  Every node of the (k M + 1)^2 lattice
 * of spacing 1/(k M) is an unknown: node g = gi + (k M + 1) gj is DoF g, so
 * n_free = (k M + 1)^2.  The smoother's patches are the vertex stars (Sec. 3:
 * the vertex and the nodes interior to its incident edges and cells,
 * 3k^2 - 3k + 1 DoFs at an interior vertex).  The operator is linear and
 * assembled at creation; stwr_nonlinear_residual gives F(U) = A U - b with
 * b = e0 (x) M U_0 on slab 0 (stwr_linear_rhs returns b), so
 * stwr_fgmres(b) is the paper's solve and stwr_newton_solve converges in one
 * step.  The coarsest level must satisfy (k M_c + 1)^2 (q + 1) <= 4096. */
#define STWR_EQ_NAVIER_STOKES 0
#define STWR_EQ_HEAT 1

/* flow = STWR_FLOW_CHORIN selects the Chorin test problem of Sec. 2 (the mode
 * arrays are then ignored and may be empty): velocity
 *   u = (-cos(pi x) sin(pi y), sin(pi x) cos(pi y)) exp(-2 pi^2 t),
 * full Dirichlet data and initial value from u, and no forcing (u with the
 * pressure -(R/4)(cos 2 pi x + cos 2 pi y) exp(-4 pi^2 t) solves the equations). */
/* flow = STWR_FLOW_CAVITY selects the lid-driven cavity of Sec. 2: velocity
 * (1, 0) on the open top side, zero on the other sides and at the two top
 * corners, zero initial velocity (the lid moves from the first slab on), no
 * forcing; there is no exact solution (stwr_velocity_l2_error then measures
 * against the boundary data). */
#define STWR_FLOW_MODES 0
#define STWR_FLOW_CHORIN 1
#define STWR_FLOW_CAVITY 2

/* Lagrange nodes of the DG(q) basis on each slab (Sec. 2 leaves them
 * unnamed).  They fix the times at which the Dirichlet data is interpolated,
 * the only place they change the discrete solution.  STWR_NODES_RADAU: right
 * Gauss-Radau points ({1}; {1/3, 1}), the slab end value is the last nodal
 * value.  STWR_NODES_GAUSS: Gauss-Legendre points ({1/2}; (3 -+ sqrt 3)/6),
 * with which the Chorin error table of Sec. 4.2 is reproduced.  Vectors hold
 * the nodal values in either case. */
#define STWR_NODES_RADAU 0
#define STWR_NODES_GAUSS 1

/* Solver options (Sec. 3 and 4.2).  stwr_default_opts fills V(2,2),
 * Chebyshev [0.25, 1.05] * lam, 10 estimation steps, FP64 smoother,
 * FGMRES(30) with rtol 1e-10 and 200 iterations, Newton rtol 1e-10, 20 steps,
 * and vcycle_graph = 1: the V-cycle is captured once into a HIP graph (on the
 * problem's stream, re-captured when the smoothers or options change) and
 * replayed for every application, with results identical to the launched
 * form; the graph's input and output vectors add 2 n_st(0) doubles to the
 * problem.  0 launches the kernels one by one. */
typedef struct {
  int32_t nu_pre, nu_post;
  double cheb_lo, cheb_hi;
  int32_t eig_steps;
  int32_t smoother_prec;       /* STWR_FP64 or STWR_FP32 patch factors and relaxation */
  int32_t gmres_restart, gmres_maxit;
  double gmres_rtol;
  int32_t newton_maxit;
  double newton_rtol;
  int32_t vcycle_graph;        /* 1: replay a captured HIP graph of the V-cycle; 0: launch */
  int32_t newton_ew;           /* 1: Eisenstat-Walker linear tolerances in Newton (see below) */
  double gmres_atol;           /* stwr_fgmres also stops once ||r|| <= gmres_atol (default 0;
                                  the paper's heat runs: rtol 1e-6, atol 1e-6) */
  int32_t time_chunks;         /* sweeps in time chunks (cyclic reduction in time, below):
                                  0 = autotuned per level (default), 1 = plain, c = c chunks */
  int32_t factor_mfma;         /* 1 (default): FP32 patch blocks of more than 64 rows are inverted
                                  by blocked Gauss-Jordan with MFMA trailing updates; 0: by the
                                  column-at-a-time register Gauss-Jordan (same pivoting rule) */
  int32_t deterministic;       /* 1: results equal bit for bit from run to run (see below);
                                  0 (default): time_chunks = 0 chooses by timing */
} stwr_solver_opts;

/* Every step of a solve runs in a fixed order: the Navier-Stokes residual
 * and Jacobian of eq. nsfem are assembled cell colour by cell colour (8
 * colours, no two cells of a colour sharing a DoF) with plain additions, the
 * patch factors and sweeps, the owner-gather of the patch corrections, the
 * reductions and the coarsest solve likewise.  The one choice made by timing
 * is time_chunks = 0 (the chunk count of each small level); deterministic = 1
 * makes it the plain sweep, and two solves then agree bit for bit.
 */

/* Time chunks (the cyclic reduction in time of Sec. 3.1, single-GPU form).
 * A patch's sweep is a forward substitution over the N slabs.  With c chunks
 * of L = ceil(N / c) slabs, every chunk is first swept from zero incoming
 * slab-end values (all chunks at once), then a small recurrence per patch
 * carries the true end values across the chunks with the chunk transfer
 * matrices T = prod (E1 A_n^{-1} E0 M_v) (built with the factors), and the
 * chunks after the first are swept again from them: 2N - L slab solves and
 * c small steps instead of N sequential slab solves, in exchange for c times
 * the parallelism.  The result equals the plain sweep up to rounding.  With
 * time_chunks = 0, stwr_setup_smoothers times 1, 2, 4, ... chunks (at least
 * two slabs each) on every level with at most 2048 patches and keeps the
 * fastest; larger levels keep the plain sweep.  The transfer matrices and end
 * values take (nv c (b^2 + 2 b)) doubles per level, b = 38 (19 for the heat
 * equation). */

/* newton_ew = 1 replaces gmres_rtol in Newton's linear solves by Eisenstat and
 * Walker's second forcing term (SIAM J. Sci. Comput. 17, 1996; the paper's
 * Chorin and cavity runs use it): eta_0 = 0.3, then
 * eta_k = (||F_k|| / ||F_{k-1}||)^((1+sqrt 5)/2), raised to eta_{k-1}^((1+sqrt 5)/2)
 * when that exceeds 0.1, at most 0.9.  Default 0. */

#define STWR_MAX_NEWTON 64
#define STWR_MAX_LEVELS 16

/* Iteration record of stwr_fgmres / stwr_newton_solve (host memory). */
typedef struct {
  int32_t newton_its;
  int32_t linear_its_total;
  int32_t linear_its[STWR_MAX_NEWTON];
  double fnorm[STWR_MAX_NEWTON + 1];      /* ||F|| before each step and at the end */
  double lambda[STWR_MAX_LEVELS];         /* last eigen-estimate per smoothed level */
  double final_rel_residual;              /* FGMRES: last relative residual */
  double setup_seconds, solve_seconds;    /* host wall clock of setup and Krylov phases */
  double linear_rel[STWR_MAX_NEWTON];     /* Newton: ||b - A dU|| / ||b|| reached by each linear solve */
} stwr_stats;

/* ---- context ---------------------------------------------------------- */
int32_t stwr_default_opts(stwr_solver_opts* opts);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  hbm_budget bounds the
 * device bytes all problems of this context may hold (0 = no bound). */
int32_t stwr_ctx_create(int32_t device, void* hip_stream, uint64_t hbm_budget, stwr_ctx** out);
int32_t stwr_ctx_destroy(stwr_ctx* ctx);
int32_t stwr_ctx_set_stream(stwr_ctx* ctx, void* hip_stream);
const char* stwr_last_error(const stwr_ctx* ctx);
/* Bytes currently held by the context's problems. */
int32_t stwr_ctx_bytes_in_use(const stwr_ctx* ctx, uint64_t* bytes);

/* Kernel timing: when enabled, the library brackets every launch of the
 * patch-sweep kernel (and of the space-time operator kernel) with HIP events
 * on the context's stream.  stwr_ctx_kernel_times synchronises the stream and
 * returns, per kernel class k (0 = patch sweep, 1 = operator apply/residual,
 * 2 = patch gather/update), the summed milliseconds and launch count since
 * the last reset; it then resets the counters.  ms and launches hold 3 entries. */
int32_t stwr_ctx_set_timing(stwr_ctx* ctx, int32_t enable);
int32_t stwr_ctx_kernel_times(stwr_ctx* ctx, double* ms, int64_t* launches);

/* Measurement aid for the roofline of the memory-bound kernels (the patch
 * sweep of Sec. 3 and the operator of eq. nsfem): the device's attainable HBM
 * read rate, reported beside the published peak.  Reads `bytes` of the
 * caller's device buffer `buf` (a multiple of 16, at least 64 MiB so that
 * caches do not serve it; not modified) with a grid-stride kernel of 16-byte
 * nontemporal loads, eight 256-thread workgroups per CU, on the context's
 * stream; one untimed launch, then `reps` launches timed with HIP events.
 * *gbs = bytes / fastest launch, in GB/s.  Allocates and frees a small
 * partial-sum buffer and synchronises the stream.  STWR_ERR_ARG on a bad
 * size, pointer or reps < 1. */
int32_t stwr_ctx_read_rate(stwr_ctx* ctx, const void* buf, uint64_t bytes, int32_t reps, double* gbs);

/* Allocate problem memory stream-ordered (hipMallocAsync/hipFreeAsync on the
 * context's stream) instead of hipMalloc/hipFree, so that freeing a finished
 * problem does not synchronise the device while other streams work. */
int32_t stwr_ctx_set_alloc_mode(stwr_ctx* ctx, int32_t stream_ordered);

/* ---- host-only queries (no device needed) ------------------------------ */
/* Device bytes stwr_problem_create would allocate (factors at the chosen
 * precision, operators, maps, Krylov and smoother workspaces). */
int32_t stwr_problem_bytes(const stwr_problem_desc* desc, const stwr_solver_opts* opts,
                           uint64_t* bytes);
/* Length n_st of the problem's level-0 space-time vectors (the solution,
 * F(U), right-hand sides): free spatial DoFs x n_slabs x (q+1), where the
 * free DoFs are 2 (2M-1)^2 + (M+1)^2 for Navier-Stokes (Taylor-Hood P2-P1,
 * boundary velocity eliminated) and (kM+1)^2 for the heat equation's P_k
 * lattice (k = degree).  Host only; STWR_ERR_ARG for an invalid descriptor. */
int32_t stwr_problem_n_st(const stwr_problem_desc* desc, int64_t* n_st);

/* Host-built structure of one mesh with M squares a side, for checking the
 * setup against closed-form counts.  out[0..11] = n_free, n_nodes_p2,
 * n_vertices, n_cells, csr_nnz, n_patches, sum_patch_dofs, max_patch_dofs,
 * interior-patch nonzeros (velocity-velocity), interior-patch nonzeros
 * (velocity-pressure), interior-patch nonzeros (pressure-velocity),
 * number of distinct patch sizes; out[12..] = histogram of patch sizes
 * 0..39 (40 entries).  out must hold 52 int64. */
int32_t stwr_mesh_info(int32_t mesh_n, int64_t* out);

/* Host-built Vanka+star patches of one Navier-Stokes level with M = mesh_n
 * squares a side and pressure degree `degree` (1: Taylor-Hood P2-P1, 2:
 * P3-P2; Sec. 3 patches, Sec. 3.1 counts), in the free numbering above (for
 * P3-P2 on its own lattices: velocity node (gi, gj) of the (3M+1)^2 lattice,
 * interior, is k = (gi-1) + (3M-1)(gj-1) with DoFs 2k and 2k+1; pressure node
 * g of the (2M+1)^2 lattice is DoF 2 (3M-1)^2 + g).  counts[0..6] = free
 * DoFs, patches (one per vertex), sum of patch sizes, CSR nonzeros, largest
 * patch, structural nonzeros of the patch of the vertex nearest the centre
 * (velocity-velocity and velocity-pressure pairs that share a cell), cells.  patch_ptr (patches + 1) and patch_dofs (sum of sizes; each patch's
 * DoFs ascending) are filled when not NULL.  Host only. */
int32_t stwr_level_patches(int32_t mesh_n, int32_t degree, int64_t* counts, int32_t* patch_ptr,
                           int32_t* patch_dofs);
/* Host-built prolongation from the mesh_n/2 level to the mesh_n level of the
 * same pressure degree (nested interpolation of each velocity component and
 * of the pressure, Sec. 3), by fine free DoF rows: counts[0..2] = fine free
 * DoFs, coarse free DoFs, nonzeros; p_ptr (fine + 1), p_col, p_val (nonzeros)
 * and inject (coarse free DoF -> fine free DoF at the same node, coarse) are
 * filled when not NULL.  mesh_n even.  Host only. */
int32_t stwr_level_transfer(int32_t mesh_n, int32_t degree, int64_t* counts, int32_t* p_ptr, int32_t* p_col,
                            double* p_val, int32_t* inject);

/* ---- problem ------------------------------------------------------------ */
int32_t stwr_problem_create(stwr_ctx* ctx, const stwr_problem_desc* desc,
                            const stwr_solver_opts* opts, stwr_problem** out);
int32_t stwr_problem_destroy(stwr_problem* p);
int32_t stwr_problem_sizes(const stwr_problem* p, int32_t level, int64_t* n_st,
                           int64_t* n_spatial_free, int32_t* n_patches);
int32_t stwr_set_opts(stwr_problem* p, const stwr_solver_opts* opts);

/* Spatial DoFs of every patch of a level (the slab blocks are (q+1) nb
 * square), patch v at nb[v]: host int32[n_patches] (Sec. 3 patches: the
 * Vanka+star patch of each vertex, or its vertex star for the heat
 * equation). */
int32_t stwr_patch_sizes(const stwr_problem* p, int32_t level, int32_t* nb);

/* Time chunks the sweeps of a level currently use (1 = the plain sweep); the
 * autotuned count is known after stwr_setup_smoothers. */
int32_t stwr_level_time_chunks(const stwr_problem* p, int32_t level, int32_t* chunks);

/* Nonlinear space-time residual F(U) of eq. nsfem (level 0), U and F of
 * length n_st(0).  Boundary values are the exact velocity at the temporal
 * nodes; the initial value is the P2 interpolant of the velocity at t = 0.
 * Heat equation: F(U) = A U - b (eq. heatfem). */
int32_t stwr_nonlinear_residual(stwr_problem* p, const double* U, double* F);

/* b = -F(0), the right-hand side of the first Newton correction; for the
 * heat equation the right-hand side of its linear system, e0 (x) M U_0 on
 * slab 0 (eq. heatfem's jump term with U_0^- the initial value).  b: device
 * vector of length n_st(0). */
int32_t stwr_linear_rhs(stwr_problem* p, double* b);

/* Space-time velocity L2 error of U against the manufactured velocity,
 * sqrt(sum_n int_{I_n} ||u - U||^2 dt) (the error measure of the paper's
 * convergence tables, Sec. 5), by the residual's quadrature rules.  U: device
 * vector of length n_st(0); err: host scalar (the call synchronises).  The
 * sum has a fixed order, so repeated calls give identical results.
 * STWR_ERR_STATE for the heat equation. */
int32_t stwr_velocity_l2_error(stwr_problem* p, const double* U, double* err);

/* Full nodal space-time vector from a free one (adds the Dirichlet values):
 * full = [ux at every P2 node][uy at every P2 node][p at every vertex], each
 * row [slab][temporal node]; P2 nodes number i + (2M+1) j on the (2M+1)^2
 * grid of the mesh, vertices i + (M+1) j.  Length
 * (2 (2M+1)^2 + (M+1)^2) N (q+1); device pointers, caller-owned.
 * STWR_ERR_STATE for the heat equation (every node is already free). */
int32_t stwr_expand(stwr_problem* p, const double* U, double* full);

/* Jacobian dF/dU at U (level 0 vector) on every level: the iterate is
 * injected to the coarse nodes and each level rediscretised; also factors
 * the coarsest level (bordered by one zero-mean pressure constraint per
 * temporal node).  Invalidates patch factors and eigen-estimates.  Heat
 * equation: rebuilds its (state-independent) operator; U is not read. */
int32_t stwr_assemble(stwr_problem* p, const double* U);

/* Copy of the assembled operator of a level (host memory): row_ptr
 * (n_free+1 int32), col (nnz int32), values (nnz * n_slabs * (q+1)^2 f64,
 * [nz][slab][a][b]), mass (nnz f64: the velocity mass matrix whose
 * -e0 e1^T (x) M couples slab n to slab n-1).  Pass NULL to query nnz only. */
int32_t stwr_get_operator(stwr_problem* p, int32_t level, int64_t* nnz, int32_t* row_ptr,
                          int32_t* col, double* values, double* mass);

/* y = A_l x  and  r = b - A_l x  (space-time operator of level l). */
int32_t stwr_apply(stwr_problem* p, int32_t level, const double* x, double* y);
int32_t stwr_residual(stwr_problem* p, int32_t level, const double* b, const double* x,
                      double* r);

/* Extract every patch block A_{v,n} = R_v J_{l,n} R_v^T of level l and
 * invert it (partial pivoting) in precision prec (STWR_FP64/STWR_FP32). */
int32_t stwr_patch_factor(stwr_problem* p, int32_t level, int32_t prec);

/* One additive waveform-relaxation Vanka application z = sum_v R_v^T A_v^{-1} R_v r:
 * per patch, forward block substitution over the slabs (eq. waveform_patch_solve). */
int32_t stwr_patch_apply(stwr_problem* p, int32_t level, const double* r, double* z);

/* stwr_patch_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, with the per-patch outputs kept in a
 * fixed 64 MiB device area of the library (one per device, resolved when the
 * first context on the device is created and held until the process ends)
 * instead of the level's own buffer.  The call allocates nothing.  The area
 * must hold the level's patch outputs, sum over patches of nb N (q+1) doubles
 * (each patch rounded up to 16 doubles); a larger level gives STWR_ERR_ARG
 * with the sizes in the message.  Every call on a device shares that
 * device's area, so calls that overlap on one device (other streams or host
 * threads) race; calls on one stream do not. */
int32_t stwr_patch_apply_noalloc(stwr_problem* p, int32_t level, const double* r, double* z);

/* lam = max real Ritz value of M^{-1} A_l after opts.eig_steps Arnoldi steps
 * from v0[i] = frac(0.6180339887498949 i) - 0.5 (normalised). */
int32_t stwr_eig_estimate(stwr_problem* p, int32_t level, double* lambda);

/* n_steps Chebyshev-accelerated relaxation sweeps on A_l x = b over [a, bnd];
 * x is updated in place.  Each sweep forms r = b - A_l x in FP64; with FP32
 * patch factors on a P2-P1 level (one time chunk) r is stored rounded to
 * FP32, the precision the FP32 patch solves take it in. */
int32_t stwr_relax(stwr_problem* p, int32_t level, const double* b, double* x,
                   int32_t n_steps, double a, double bnd);

/* rc = R rf (fine_level -> fine_level+1);  xf += P ec. */
int32_t stwr_restrict(stwr_problem* p, int32_t fine_level, const double* rf, double* rc);
int32_t stwr_prolong_add(stwr_problem* p, int32_t fine_level, const double* ec, double* xf);

/* Exact solve on the coarsest level; x has zero-mean pressure per temporal
 * node (Navier-Stokes; the heat equation's slab blocks need no border). */
int32_t stwr_coarse_solve(stwr_problem* p, const double* b, double* x);

/* Factor every smoothed level at opts.smoother_prec and estimate lam on each. */
int32_t stwr_setup_smoothers(stwr_problem* p);

/* One V-cycle of Alg. 1 on level 0 with zero initial guess: x = V(b). */
int32_t stwr_vcycle(stwr_problem* p, const double* b, double* x);

/* FGMRES(restart) on A_0 x = b, x starting at 0, right-preconditioned by one
 * V-cycle, constant pressure projected out of each preconditioned vector
 * (Navier-Stokes).  Stops when ||r|| <= max(gmres_rtol ||b||, gmres_atol);
 * STWR_ERR_NOT_CONVERGED if gmres_maxit iterations do not get there. */
int32_t stwr_fgmres(stwr_problem* p, const double* b, double* x, stwr_stats* stats);

/* Newton's method from the U given (zero = the standard start), in place:
 * assemble, factor, estimate, FGMRES, U += dU, until ||F|| <= rtol ||F_0||.
 * Full steps; STWR_ERR_NOT_CONVERGED after newton_maxit steps, or as soon as
 * ||F|| exceeds 100 ||F_0|| (divergence), with stats filled either way. */
int32_t stwr_newton_solve(stwr_problem* p, double* U, stwr_stats* stats);

/* Subtract the mean pressure per (slab, temporal node) from x (level l). */
int32_t stwr_project_pressure(stwr_problem* p, int32_t level, double* x);

/* ---- serving: continuous batching of independent solves ------------------
 * A server owns n_slots workers, each with its own non-blocking HIP stream on
 * `device`.  Submitted requests wait in FIFO order and are admitted when a
 * worker is free and the request's device bytes (stwr_problem_bytes plus its
 * solution vector) fit in hbm_budget minus the bytes of the solves in flight
 * (0 = no bound); a request larger than the whole budget completes at once
 * with STWR_ERR_BUDGET.  An admitted request is created, solved by
 * stwr_newton_solve from the zero start, its solution copied to `host_out`
 * (n_st doubles as stwr_problem_n_st gives them, for either equation, or
 * NULL to discard), and its memory released, so solves of
 * different sizes overlap on the device.  Times are seconds on the server's
 * steady clock (stwr_server_now). */
typedef struct stwr_server stwr_server;

typedef struct {
  int64_t id;
  int32_t status;              /* stwr_status of the solve */
  int32_t newton_its, linear_its;
  int32_t slot;                /* worker that ran it (-1 if rejected) */
  double submit_time, start_time, end_time;
  double fnorm_ratio;          /* final ||F|| / ||F_0|| */
  uint64_t bytes;              /* device bytes reserved for it */
} stwr_result;

int32_t stwr_server_create(int32_t device, int32_t n_slots, uint64_t hbm_budget,
                           stwr_server** out);
/* desc/opts are copied; host_out must stay valid until the result is polled. */
int32_t stwr_server_submit(stwr_server* s, const stwr_problem_desc* desc,
                           const stwr_solver_opts* opts, double* host_out, int64_t* id_out);
/* Move up to max_results finished results into `results`; *n_out = count. */
int32_t stwr_server_poll(stwr_server* s, stwr_result* results, int32_t max_results,
                         int32_t* n_out);
/* Block until every submitted request has finished or timeout_s elapses
 * (returns STWR_ERR_STATE on timeout). */
int32_t stwr_server_wait(stwr_server* s, double timeout_s);
int32_t stwr_server_now(const stwr_server* s, double* t);
/* Finishes the requests in flight, drops the queued ones, joins the workers. */
int32_t stwr_server_destroy(stwr_server* s);

/* ---- batched solves: many problems in shared launches ------------------
 * A batch advances many independent Navier-Stokes solves together on its
 * context's stream, each exactly as stwr_newton_solve would with FP32 patch
 * factors and sweeps and the plain sweep in time (time_chunks = 1): the patch
 * systems are independent across patches and so across problems (eq.
 * waveform_patch_solve), so every relaxation sweep covers the patches of
 * every problem at that multigrid depth in one persistent launch per
 * temporal-node count, and every patch factorization all levels of all
 * problems at the start of a Newton step in one persistent launch per block
 * class.  The patches (sweep) or blocks (factorization) a workgroup takes at
 * a time are chosen per class by timing the candidates on the batch.  With
 * use_graph = 1 the batched V-cycle is captured into a HIP graph and replayed
 * while the set of problems in their Krylov phase (and their Newton steps) is
 * unchanged.  A problem's result equals its solve alone with the same
 * options up to rounding (the operations are the same, in the same order).
 *
 * stwr_batch_add creates the problem at once on the batch's context
 * (STWR_ERR_BUDGET if it does not fit the context's HBM budget; nothing is
 * then kept) and starts it at the next step.  It must be a Navier-Stokes
 * P2-P1 problem with at least two levels and smoother_prec = STWR_FP32; every
 * problem of a batch has the same nu_pre and nu_post (the first fixes them).
 * host_out: n_st doubles of host memory for the solution (or NULL), written
 * when the problem finishes and valid once its result is polled.
 * stwr_batch_step: one step, i.e. one FGMRES iteration of every problem in
 * its Krylov phase, after the Newton bookkeeping, assembly, factorization and
 * eigen-estimates of those starting a Newton step; *n_live = problems not yet
 * finished.  Finished problems are released and their results (status,
 * iterations, times on the batch's clock in seconds) queued for
 * stwr_batch_poll.  stwr_batch_info fills out[0..10]: steps, graph captures,
 * V-cycles, sweep launches, factorization launches, sweep tiles (one and two
 * temporal nodes; 0 = not chosen yet), factorization tiles (three classes),
 * live problems. */
typedef struct stwr_batch stwr_batch;

int32_t stwr_batch_create(stwr_ctx* ctx, int32_t use_graph, stwr_batch** out);
int32_t stwr_batch_add(stwr_batch* b, const stwr_problem_desc* desc, const stwr_solver_opts* opts,
                       double* host_out, int64_t* id_out);
int32_t stwr_batch_step(stwr_batch* b, int32_t* n_live);
int32_t stwr_batch_poll(stwr_batch* b, stwr_result* results, int32_t max_results, int32_t* n_out);
int32_t stwr_batch_info(const stwr_batch* b, int64_t* out);
int32_t stwr_batch_destroy(stwr_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* STWR_H */
