/*
 * ldgs.h -- C ABI of the LDG-Stokes multigrid library for MI355X (gfx950).
 *
 * The library solves the discrete (multi-phase, optionally unsteady) Stokes
 * system of Saye, "Fast multigrid solution of high-order accurate multi-phase
 * Stokes problems": the LDG saddle-point operator of eq. (blockform) /
 * eq. (stokessystem) on a uniform Cartesian grid of the unit square or cube,
 * with the V-cycle of Algorithm 1 (element-block Gauss-Seidel smoothing in a
 * fixed multicolour order, injection prolongation, restriction by its
 * transpose, an eigen-decomposition pseudo-inverse at the bottom) and the
 * operator-coarsened hierarchy of Algorithms 2 and 3.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an ldgs_status and never throws.  On error the
 *    context (if any) keeps a message readable with ldgs_last_error().
 *  - Vectors b and x are caller-owned FP64 device pointers of length
 *    ldgs_num_dofs(), element-lexicographic (axis 0 fastest); within an
 *    element field-major (u_1 .. u_d, p); within a field the coefficients of
 *    the orthonormal tensor-product Legendre basis
 *      phi_a(x) = h^{-d/2} prod_k l_{a_k}((x_k - x_{E,k}) / h),
 *      l_m(xi) = sqrt(2m+1) P_m(2 xi - 1),  a = sum_k a_k (p+1)^k.
 *    Pointers must be 8-byte aligned and must not alias unless stated.
 *  - All device work is ordered on the stream given in ldgs_problem; calls
 *    that return host-visible results (norms, convergence) synchronise it.
 *  - A context is not thread-safe.  Distinct contexts are independent.
 */
#ifndef LDGS_H
#define LDGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LDGS_OK = 0,
  LDGS_E_ARG = 1,            /* invalid argument (null pointer, bad size, bad enum) */
  LDGS_E_UNSUPPORTED = 2,    /* a valid but unimplemented combination */
  LDGS_E_NOMEM = 3,          /* host or device allocation failed */
  LDGS_E_HIP = 4,            /* a HIP runtime call failed */
  LDGS_E_SINGULAR_BLOCK = 5, /* an element block A_EE is numerically singular */
  LDGS_E_COLORING = 6,       /* the colouring couples two elements of one colour */
  LDGS_E_NOT_CONVERGED = 7,  /* tolerance not reached within maxit, or divergence */
  LDGS_E_NONFINITE = 8       /* a NaN or Inf appeared in a residual norm */
} ldgs_status;

/* gamma of eq. (govern1): 0 standard form -mu lap u, 1 viscous-stress form. */
typedef enum { LDGS_STANDARD = 0, LDGS_VISCOUS_STRESS = 1 } ldgs_form;

/* Boundary condition of one axis (both sides); eq. (govern3).  Stress
 * boundaries are declared but return LDGS_E_UNSUPPORTED. */
typedef enum { LDGS_PERIODIC = 0, LDGS_DIRICHLET = 1, LDGS_STRESS = 2 } ldgs_bc;

/* Multicolour ordering of the block Gauss-Seidel smoother (section 3).
 * Colour of element i = (i_0, .., i_{d-1}):
 *   RED_BLACK  sum_k i_k mod 2                 (2 colours)
 *   PARITY     sum_k (i_k mod 2) 2^k           (2^d colours)
 *   MOD3       sum_k (i_k mod 3) 3^k           (3^d colours)
 * AUTO picks the first of these that is proper for the operator's stencil;
 * a colouring that couples two same-coloured elements gives LDGS_E_COLORING.
 * Colours are swept in increasing order in pre- and post-smoothing. */
typedef enum { LDGS_COLOR_AUTO = 0, LDGS_COLOR_RED_BLACK = 1, LDGS_COLOR_PARITY = 2,
               LDGS_COLOR_MOD3 = 3 } ldgs_coloring;

/* Arithmetic of the V-cycle.  FP64: everything in double.  FP32: smoother,
 * residuals and transfers in float with float block inverses (computed in
 * double); bottom solve in double.  FP32_BF16BLK: as FP32 but the block
 * inverses are stored as bfloat16. */
typedef enum { LDGS_V_FP64 = 0, LDGS_V_FP32 = 1, LDGS_V_FP32_BF16BLK = 2 } ldgs_vprec;

/* Outer iteration of ldgs_solve.  STATIONARY: x <- V(b, x).  IR: r = b - A x
 * in FP64, x += V(r, 0).  FGMRES: flexible GMRES(m), right-preconditioned by
 * one V-cycle from zero, FP64 Arnoldi with modified Gram-Schmidt (stores 2m+1
 * vectors).  GMRES: GMRES(m) right-preconditioned by the same V-cycle taken
 * as a fixed operator M (stores m+2 vectors; x += M (V_m y) at the end of
 * each restart cycle, one extra V-cycle); the V-cycle from zero is linear,
 * so this is exact for the FP64 cycle and holds to the cycle's rounding in
 * FP32. */
typedef enum { LDGS_STATIONARY = 0, LDGS_IR = 1, LDGS_FGMRES = 2, LDGS_GMRES = 3 } ldgs_outer;

/* Scalar coefficient fields (viscosity mu, density rho). */
typedef enum {
  LDGS_FIELD_CONST = 0,         /* params[0] = c */
  LDGS_FIELD_SINSIN = 1,        /* a + b prod_k sin(2 pi k x_k): params = {a, b, k} */
  LDGS_FIELD_LOGNORMAL_RFF = 2, /* 10^{g}, g = sqrt(2/K) sum_m cos(k_m . x + phi_m):
                                   params = {k_1 (d values) .. k_K, phi_1 .. phi_K},
                                   nparams = K (d + 1) */
  LDGS_FIELD_PHASE_CONST = 3,   /* params[0] in phase 1, params[1] in phase 2 */
  LDGS_FIELD_CALLBACK = 4       /* values from fn */
} ldgs_field_kind;

/* Level set describing the phases.  NONE: one phase.  BOX: phase 1 is the
 * open box (params[0], params[1])^d, phase 2 its complement; box faces must
 * lie on element faces of the coarsest grid.  CIRCLE (2D, Dirichlet walls;
 * steady, or unsteady (delta > 0) with a density constant per phase, the
 * pressure penalty of eq. (taugeneral) and Algorithm 3's coarsening): phase 1
 * is the disk |x - levelset_centre| < params[0], phase 2 the
 * rest of the square; the circle cuts the grid's cells and the mesh is an
 * implicitly defined one (section 5, "Curved domain geometry"): cut cells
 * carry quadrature of their own (q_cut Gauss points per piece), pieces below
 * a quarter of a cell are merged into a neighbour of their phase, the
 * interphase penalty prefactor defaults to 8 and the intraphase one is
 * tau_u_intra_C (appendix A), coarse levels agglomerate same-phase elements
 * (section 3, "Mesh hierarchy") and every level is held as explicit element
 * blocks, smoothed in greedy colour order.  Only the FP64 and FP32 V-cycles
 * are built; the learned correction is not available. */
/* DISK: the domain itself is the disk |x - levelset_centre| < params[0]
 * inside the unit square (a curved domain, section 5): the mesh is the
 * implicitly defined one of CIRCLE without phase 2, and the circle is a
 * velocity Dirichlet boundary (data from g_dirichlet at its points, normal
 * pointing out of the disk); one phase, the same restrictions as CIRCLE. */
typedef enum {
  LDGS_LEVELSET_NONE = 0,
  LDGS_LEVELSET_BOX = 1,
  LDGS_LEVELSET_CIRCLE = 2,
  LDGS_LEVELSET_DISK = 3
} ldgs_levelset_kind;

/* Batched host callback: evaluate at n points x (n x d, row-major).  phase[i]
 * is the phase (1 or 2) of the element owning point i; normal (n x d) is the
 * face normal where the quantity lives on a face (NULL in volumes).  Writes
 * n x ncomp values to out. */
typedef void (*ldgs_eval_fn)(int64_t n, const double* x, const int* phase,
                             const double* normal, double* out, void* user);

typedef struct {
  int kind;                 /* ldgs_field_kind */
  const double* params;     /* host, read during ldgs_setup only */
  int64_t nparams;
  ldgs_eval_fn fn;          /* for LDGS_FIELD_CALLBACK */
  void* user;
} ldgs_field;

typedef struct {
  int dim;                  /* d in {2, 3} */
  int n;                    /* elements per axis, a power of two */
  int degree;               /* p in {1, 2, 3} (Q_p, same degree for u and p) */
  int form;                 /* ldgs_form (gamma) */
  int bc[3];                /* ldgs_bc per axis, both sides; LDGS_STRESS (eq. govern3,
                               u-hat = u- and sigma-hat = h n on the wall, eq. ustarflux
                               and eq. qstarflux) must be given on every axis; the
                               trivial kernel is then the rigid motions of the velocity */
  ldgs_field mu;            /* viscosity > 0 */
  ldgs_field rho;           /* density >= 0, used when delta > 0 */
  double delta;             /* > 0: unsteady operator (1/delta) M_rho + A of eq. (timedep2) */
  int levelset_kind;        /* ldgs_levelset_kind */
  double levelset_params[2];
  double tau;               /* pressure penalty prefactor of eq. (taueqn); <= 0: Table 1 */
  double tau0;              /* unsteady prefactor of eq. (taugeneral); <= 0: 0.5 p */
  double tau_u_bdry_C;      /* tau_u,boundary = C p mu^- / h; <= 0: 10 */
  double tau_u_inter_C;     /* tau_u,interphase = C p min(mu) / h; <= 0: 3 (8 on
                               implicitly defined meshes) */
  int nu1, nu2;             /* pre-/post-smoothing sweeps; <= 0: 3 */
  int coarsest_n;           /* bottom grid size; <= 0: 4 (2D), 2 (3D) */
  int coloring;             /* ldgs_coloring */
  int vprec;                /* ldgs_vprec used by ldgs_vcycle / ldgs_solve */
  int build_precisions;     /* bit mask of extra V-cycle precisions to build
                               (bit k = ldgs_vprec k); 0: only vprec */
  int diag_scaling;         /* nonzero: (alpha, beta) scaling of the multi-phase section */
  int host_only;            /* nonzero: build the host-side operator data only (setup
                               validation without a GPU); device entry points then
                               return LDGS_E_UNSUPPORTED and ldgs_assemble_rhs writes
                               to a host pointer */
  void* hip_stream;         /* hipStream_t the context works on.  NULL: the
                               library creates a stream of its own (the legacy
                               null stream cannot be captured into a graph) and
                               orders it, at every call, after the work queued
                               on the null stream before the call, and the null
                               stream after the work of the call */
  /* Device allocator for all storage of the context (operator data, block
   * inverses, work vectors, Krylov basis), e.g. a framework's caching
   * allocator, so that the caller stays the owner of device memory.
   * dev_alloc(bytes, alloc_user) returns a 256-byte aligned device pointer or
   * NULL (then the call that needed it fails with LDGS_E_NOMEM);
   * dev_free(ptr, alloc_user) receives every block back in ldgs_destroy,
   * after the context's stream has drained.  Both NULL: hipMalloc/hipFree.
   * Giving only one of them is LDGS_E_ARG.  The callbacks are called from
   * the thread that calls into the library, never during graph capture. */
  void* (*dev_alloc)(size_t bytes, void* alloc_user);
  void (*dev_free)(void* ptr, void* alloc_user);
  void* alloc_user;
  double levelset_centre[3];  /* LDGS_LEVELSET_CIRCLE: centre of the circle */
  double tau_u_intra_C;       /* tau_u,0 = C p mu / h on intraphase faces of implicitly
                                 defined meshes (appendix A gives 0.5 for them); Cartesian
                                 grids use 0 */
  int q_cut;                  /* Gauss points per piece in cut-cell quadrature; <= 0: 8 */
} ldgs_problem;

/* Data of the right-hand side, eq. (govern1)-(govern3).  Each callback may be
 * NULL (meaning zero).  ncomp: f d, f_div 1, g_dirichlet d, g_jump d, h_jump d,
 * h_stress d.  g_jump / h_jump are the jumps [u] and [sigma n] on interphase
 * faces, normal from phase 1 into phase 2, phase[] giving the phase-1 side.
 * h_stress is the stress data h = sigma n on stress walls (n outward; it
 * enters through the vector J_h of the appendix on the LDG construction). */
typedef struct {
  ldgs_eval_fn f, f_div, g_dirichlet, g_jump, h_jump, h_stress;
  void* user;
} ldgs_rhs_data;

typedef struct {
  int iters;                /* outer iterations (V-cycles) performed */
  int fallback_events;      /* learned correction switched off (0 otherwise) */
  double relres;            /* final ||b - A x||_2 / ||b||_2, FP64, recomputed */
  double rho_measured;      /* geometric mean residual reduction per iteration */
  double t_solve_s;         /* wall time of the solve */
  double* history;          /* caller-owned host array, or NULL */
  int history_cap;
  int history_len;          /* relres after each iteration, history[0] = 1 */
} ldgs_info;

typedef struct ldgs_ctx ldgs_ctx;

/* Build every level (operator coarsening, Algorithms 2/3), the colouring,
 * the factorised diagonal blocks of each smoothed level (explicit FP64
 * inverses of the equilibrated LU, then cast) and the bottom pseudo-inverse.
 * Synchronises.  *out receives a new context owned by the caller. */
ldgs_status ldgs_setup(const ldgs_problem* prob, ldgs_ctx** out);

/* Number of unknowns N = n^d (d+1) (p+1)^d. */
ldgs_status ldgs_num_dofs(const ldgs_ctx* ctx, int64_t* ndof);

/* b of eq. (stokessystem): momentum rows int f_i phi - sum_j G_j^T M_mu
 * (J_g,ij + gamma J_g,ji) + J_h,i + penalty data; constraint rows int f phi +
 * J_{g.n} (appendix A).  Assembled on the host, copied to b_dev.  Synchronises. */
ldgs_status ldgs_assemble_rhs(ldgs_ctx* ctx, const ldgs_rhs_data* data, double* b_dev);

/* y = A x (FP64, unscaled operator), matrix-free.  x and y must not alias. */
ldgs_status ldgs_apply(ldgs_ctx* ctx, const double* x_dev, double* y_dev);

/* r = b - A x (FP64); if norm2_host is non-NULL, *norm2_host = ||r||_2
 * (synchronises).  r may be NULL when only the norm is wanted. */
ldgs_status ldgs_residual(ldgs_ctx* ctx, const double* b_dev, const double* x_dev,
                          double* r_dev, double* norm2_host);

/* One V-cycle of Algorithm 1 in place on x, in the context's precision. */
ldgs_status ldgs_vcycle(ldgs_ctx* ctx, const double* b_dev, double* x_dev);

/* Solve A x = b to ||b - A x|| <= tol ||b|| from the x given (use zeros).
 * b is first projected onto range(A) (its components along the trivial
 * kernel are removed, in place).  maxit bounds the outer iterations;
 * fgmres_m is the restart length.  use_learned (outer = LDGS_IR or
 * LDGS_FGMRES; needs ldgs_set_learned) replaces each V-cycle result z = V(v)
 * by z + w dx, dx the network's correction of the residual r' = v - A z the
 * cycle leaves and w = <r', A dx> / ||A dx||^2 the minimal-residual step, both
 * in the cycle's precision and variables (one extra finest-level apply), so
 * that the corrected step never leaves a larger residual in those variables.
 * FGMRES takes the corrected result as its preconditioned direction.  Under
 * LDGS_IR a guard also applies: the first two iterations are plain and give
 * rho_plain = (||r_2|| / ||r_0||)^(1/2); the correction is switched off for
 * the rest of the solve when an iteration's reduction
 * c_k = ||r_k|| / ||r_{k-1}|| exceeds 1, or exceeds 1.1 rho_plain twice in a
 * row, and that iteration is redone without it (info->fallback_events counts
 * this).  info may be NULL.  Synchronises. */
ldgs_status ldgs_solve(ldgs_ctx* ctx, double* b_dev, double* x_dev, double tol, int maxit,
                       int outer, int fgmres_m, int use_learned, ldgs_info* info);

/* Number of V-cycles captured into HIP graphs so far (one per precision,
 * zero-guess flag and timing stride; each is replayed on later cycles).  0
 * when graphs are off (environment variable LDGS_GRAPH=0 at setup) or when a
 * capture failed, in which case the cycles are launched directly. */
ldgs_status ldgs_graph_count(const ldgs_ctx* ctx, int* n_graphs);

/* Convergence rate rho of eq. (rho) (section 4): GMRES without restarts,
 * left-preconditioned by V = one V-cycle from a zero guess in the context's
 * precision, on V A x = V b with b = 0, from the caller's x0 (FP64 device
 * vector, not modified), until ||V A x_k|| <= reduction ||V A x_0|| (the
 * paper uses 1e-8) or maxit (<= 1000) iterations; then
 *   rho = (||V A x_n|| / ||V A x_0||)^(1/n),  n iterations.
 * The Arnoldi basis (maxit + 2 vectors of N FP64 entries) is allocated on
 * first use and kept.  history (host, may be NULL) receives the ratios
 * ||V A x_k|| / ||V A x_0||, k = 0..n, up to history_cap entries.  Returns
 * LDGS_E_NOT_CONVERGED (rho and iters still set) if the reduction was not
 * reached.  Synchronises. */
ldgs_status ldgs_gmres_rho(ldgs_ctx* ctx, const double* x0_dev, double reduction, int maxit, double* rho,
                           int* iters, double* history, int history_cap);

/* Switch the precision used by ldgs_vcycle / ldgs_solve among those built. */
ldgs_status ldgs_set_vprec(ldgs_ctx* ctx, int vprec);

/* ---- Learned post-smoothing correction ---------------------------------
 * Not part of the paper's method; an optional extra step after the V-cycle.
 * Per finest element E a small network maps the 3^d patch of elements around
 * E (offsets in {-1,0,1}^d, axis 0 fastest; zero beyond a non-periodic wall,
 * wrapped on periodic axes) to a correction of x_E:
 *   z_F  = n_b residual coefficients of F divided by the global RMS s_f of
 *          their field (velocity or pressure), then log10 of F's mean
 *          viscosity: n_b + 1 channels per patch element;
 *   h1   = relu(W1 z + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3;
 *   dx_E = y * s_f * c_f per coefficient, f the coefficient's field.
 * Hidden width H = 16.  Inference and training run in bfloat16 (inputs,
 * weights, hidden activations; round to nearest even) on matrix cores with
 * FP32 accumulation; biases are FP32.
 *
 * Flat parameter layout (FP32, host): W1 [H][3^d][n_b+1] | b1 [H] |
 * W2 [H][H] | b2 [H] | W3 [n_b][H] | b3 [n_b];
 * nparams = H 3^d (n_b+1) + 2H + H^2 + n_b H + n_b. */
typedef struct {
  int dim, degree, hidden;  /* must match the context; hidden = 16 */
  const float* params;      /* host, flat layout above (copied) */
  int64_t nparams;
  double c_vel, c_pre;      /* output scales c_f (RMS of e / s_f on training data) */
} ldgs_net;

/* Load (net non-NULL) or remove (NULL) the correction network. */
ldgs_status ldgs_set_learned(ldgs_ctx* ctx, const ldgs_net* net);

/* dx = the network's correction for residual r (finest level, unscaled,
 * FP64 device vectors of N entries).  Asynchronous on the context stream.
 * LDGS_E_ARG without a loaded network. */
ldgs_status ldgs_learned_correction(ldgs_ctx* ctx, const double* r_dev, double* dx_dev);

/* Training pairs from plain V-cycles (the context's precision) on
 * A x = A x*, from x = 0: after cycle k (k < ncycles) with iterate x_k,
 *   r = b - A x_k and e = x* - x_k with the trivial kernel removed,
 * written as crops.  Crop c of cycle k has origin origins[(k*ncrops + c)*d + j]
 * (host ints; 0 <= origin_j, and origin_j + C <= n on non-periodic axes):
 *   feat [k][c][(C+2)^d][CHP] bf16: channels of the crop and a one-element
 *        halo (layout of the network input, CHP = roundup(n_b+1, 8), unused
 *        channels zero);
 *   targ [k][c][C^d][n_b] bf16: e / s_f on the crop.
 * C is a power of two with 4 <= C <= n.  stats_host (may be NULL) receives
 * per cycle (s_vel, s_pre, RMS(e_vel)/s_vel, RMS(e_pre)/s_pre).  x* is a
 * device FP64 vector; feat and targ device arrays.  Synchronises. */
ldgs_status ldgs_learned_collect(ldgs_ctx* ctx, const double* xstar_dev, int ncycles, int crop, int ncrops,
                                 const int* origins, uint16_t* feat_dev, uint16_t* targ_dev,
                                 double* stats_host);

/* Training on crops written by ldgs_learned_collect: Adam (Kingma and Ba) on
 * FP32 master weights; forward and backward in bfloat16 with FP32
 * accumulation; loss = mean over the batch of (y - targ / c_f)^2. */
typedef struct {
  void* hip_stream;         /* NULL = default stream */
  int dim, degree, hidden, crop, ncrops;
  const uint16_t* feat;     /* device, [ncrops][(C+2)^d][CHP] */
  const uint16_t* targ;     /* device, [ncrops][C^d][n_b] */
  double c_vel, c_pre;
  int batch, steps;
  const int* order;         /* host [steps][batch] crop indices */
  float lr, beta1, beta2, eps;
} ldgs_train_args;

/* params: in/out, flat layout (host FP32).  loss_out: host [steps], the
 * batch loss before each update (may be NULL).  grad0_out: host, flat
 * layout, the gradient of the first step (may be NULL).  Synchronises.
 * Errors are reported through ldgs_last_error(NULL). */
ldgs_status ldgs_learned_train(const ldgs_train_args* args, float* params, double* loss_out, float* grad0_out);

/* Size of the fixed device workspace of ldgs_learned_train_noalloc (per GPU). */
#define LDGS_TRAIN_WORKSPACE_BYTES ((size_t)4 << 20)

/* ldgs_learned_train for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation on the same kernels, with every device
 * buffer of the run (FP32 parameters and their BF16 copy, gradient, Adam
 * moments, per-step losses, batch order) carved from a fixed workspace of
 * LDGS_TRAIN_WORKSPACE_BYTES that the library holds on each GPU it runs on
 * until the process ends.  It calls no device allocator.  The caller still
 * passes the crops (device) and the host arrays of ldgs_learned_train.  A run
 * needs about 5 * 4 * (padded parameter count) bytes plus
 * 4 * steps * batch + 8 * steps; one that needs more than the workspace
 * returns LDGS_E_ARG before any device work.  Every call re-initialises what
 * it uses (the gradient, moments and losses are cleared by kernels), so
 * results do not depend on earlier calls.  All calls on one GPU share its
 * workspace: calls that overlap in time on one GPU (several host threads, or
 * streams that run concurrently) race and must be serialised by the caller.
 * Synchronises args->hip_stream.  Errors through ldgs_last_error(NULL). */
ldgs_status ldgs_learned_train_noalloc(const ldgs_train_args* args, float* params, double* loss_out,
                                       float* grad0_out);

/* Remove from v its components along the trivial kernel (constant pressure,
 * and constant velocity for periodic steady problems), in place. */
ldgs_status ldgs_project_kernel(ldgs_ctx* ctx, double* v_dev);

/* ---- Stage entry points (one step of the hot path on one level) --------
 * Level 0 is the finest.  Level vectors have NE_l (d+1)(p+1)^d FP64 entries
 * in the layout above, NE_l = n_l^d on Cartesian grids and the element count
 * of ldgs_level_elements on implicitly defined meshes.  They operate on the
 * operator of that level as used by the V-cycle (diagonally scaled when
 * diag_scaling is on) in FP64. */

/* Grid size n_l (background cells per axis), number of levels and colours. */
ldgs_status ldgs_level_info(const ldgs_ctx* ctx, int level, int* n_l, int* n_levels, int* n_colours);

/* Number of elements NE_l of level `level` (n_l^d on Cartesian grids; on an
 * implicitly defined mesh the cut, merged and agglomerated elements of
 * section 3, "Mesh hierarchy", numbered by (host cell, phase)).  Works on
 * host-only contexts.  Errors: LDGS_E_ARG for a null pointer or a level out
 * of range. */
ldgs_status ldgs_level_elements(const ldgs_ctx* ctx, int level, int64_t* ne);

/* Number of stored nb x nb element blocks A_EF of level `level` of an
 * implicitly defined mesh (the block rows of section 3's Gauss-Seidel
 * update; the diagonal blocks included).  Works on host-only contexts.
 * Errors: LDGS_E_ARG for a null pointer or a level out of range,
 * LDGS_E_UNSUPPORTED on Cartesian grids (no explicit blocks). */
ldgs_status ldgs_level_blocks(const ldgs_ctx* ctx, int level, int64_t* nblocks);

/* *shared = 1 when every diagonal block of level `level` is the same matrix
 * (constant viscosity and density, a periodic grid, no interphase faces: the
 * operator is translation invariant), so that its colour passes hold one
 * inverse for the level instead of one per element; 0 otherwise (and on the
 * coarsest level, which is not smoothed).  Setting the environment variable
 * LDGS_SHARED_INVERSE=0 before setup turns this off.  Works on host-only
 * contexts.  Errors: LDGS_E_ARG for a null pointer or a level out of range. */
ldgs_status ldgs_level_shared_inverse(const ldgs_ctx* ctx, int level, int* shared);

/* One colour pass of block Gauss-Seidel on level `level`: for every element E
 * of colour `colour`, x_E += A_EE^{-1} (b - A x)_E, all from the x at entry. */
ldgs_status ldgs_level_smooth_colour(ldgs_ctx* ctx, int level, int colour,
                                     const double* b_dev, double* x_dev);

/* The same colour pass in a float V-cycle (vprec FP32 or FP32_BF16BLK): b and x
 * are float device vectors of the level, in the scaled variables of that
 * cycle when diag_scaling is on. */
ldgs_status ldgs_level_smooth_colour_f32(ldgs_ctx* ctx, int level, int colour, int vprec,
                                         const float* b_dev, float* x_dev);

/* r_c = I^T (b - A_l x) on level `level` (< bottom); r_c has level+1 size. */
ldgs_status ldgs_level_residual_restrict(ldgs_ctx* ctx, int level, const double* b_dev,
                                         const double* x_dev, double* rc_dev);

/* x += I x_c, injection from level+1 to level. */
ldgs_status ldgs_level_prolong_add(ldgs_ctx* ctx, int level, const double* xc_dev, double* x_dev);

/* Bottom solve x = P b, P = D (D A_c D)^+ D with D = |diag A_c|^{-1/2}: the
 * eigendecomposition of the equilibrated bottom operator with its k0
 * smallest-magnitude eigenvalues snapped to zero (k0 = dimension of the
 * trivial kernel), applied in FP64 with one step of iterative refinement.
 * Solves A_c x = b for b in range(A_c). */
ldgs_status ldgs_bottom_solve(ldgs_ctx* ctx, const double* b_dev, double* x_dev);

/* y = A_l x on level `level`. */
ldgs_status ldgs_level_apply(ldgs_ctx* ctx, int level, const double* x_dev, double* y_dev);

/* The FP64 inverse of the diagonal block A_EE of element E on `level` (the
 * equilibrated-LU inverse that the smoother streams), row-major nb*nb doubles
 * written to a host array. */
ldgs_status ldgs_level_block_inverse(ldgs_ctx* ctx, int level, int64_t element, double* inv_host);

/* y = A_l x on `level` evaluated by the host implementation of the operator
 * that setup uses for the bottom matrix and the right-hand side (host arrays).
 * For validating the setup; the solver never calls it. */
ldgs_status ldgs_host_level_apply(ldgs_ctx* ctx, int level, const double* x_host, double* y_host);

/* The bottom solve matrix P above (row-major N_c x N_c doubles, host array)
 * and the eigenvalues of the equilibrated bottom operator (N_c doubles, in no
 * particular order); either pointer may be NULL.  *nc receives N_c. */
ldgs_status ldgs_bottom_info(ldgs_ctx* ctx, int64_t* nc, double* pinv_host, double* eig_host);

/* Timing of the finest-level colour passes.  ldgs_profile(ctx, k) with k > 0
 * records a HIP event pair on the library's stream around every k-th sweep of
 * level 0, i.e. around all colour passes of that sweep, launched back to back
 * (sweeps whose passes all evaluate the operator: the sweep that starts from a
 * zero guess is not timed); k = 0 turns it off.  Each pair adds a little host
 * and queue work, so a stride above 1 keeps the timed solve close to an
 * untimed one.  ldgs_profile_read synchronises, returns the summed time (ms)
 * and the number of colour passes it covers since the last read, and clears
 * them.  While timing is on, V-cycles are launched directly instead of
 * being replayed from graphs (events recorded inside a captured graph cannot
 * be timed from the host). */
ldgs_status ldgs_profile(ldgs_ctx* ctx, int enable);
ldgs_status ldgs_profile_read(ldgs_ctx* ctx, double* total_ms, int64_t* launches);

const char* ldgs_status_str(ldgs_status s);
/* Message of the context's last error; with ctx = NULL, the message of the
 * calling thread's last failed ldgs_setup. */
const char* ldgs_last_error(const ldgs_ctx* ctx);

/* Free all device and host storage of the context.  NULL is allowed. */
ldgs_status ldgs_destroy(ldgs_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LDGS_H */
