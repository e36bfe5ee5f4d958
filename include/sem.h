/*
 * sem.h -- C ABI of the MI355X (gfx950) spectral-element pressure-Poisson solver.
 *
 * Problem (paper Secs. 3.1-3.2, eqs. poissonp / bcpd / bcpdneu, read in the same-stage symmetric
 * form): find p with  -lap p = f  in the sigma-mapped fluid domain (Sec. 2.2, eq. sigtrans),
 * p = g_D on the free surface (top), n . grad p = g_N on walls and bottom.  Discretised with
 * nodal GLL spectral elements (Sec. 4, eqs. fglobal / flocal / flocal2 with GLL collocation)
 * and solved by geometric p-multigrid (Sec. 5: order hierarchy eq. gridcoars read as
 * ceil(P/2), interpolation/restriction of Sec. 5.2, V-cycle of Sec. 5) inside an FP64
 * flexible CG or preconditioned defect-correction loop (Sec. 5.4).
 *
 * Conventions common to every call
 *  - Global vectors are FP64, contiguous, on the context's device, length n_global:
 *      2D  g = ix (Nz P + 1) + iz,          ix in [0, Nx P], iz in [0, Nz P]
 *      3D  g = (ix (Ny P + 1) + iy)(Nz P + 1) + iz
 *    (vertical/sigma index fastest; iz = Nz P is the free surface).
 *  - Device pointers are caller-owned; the library never frees or retains them.  Host arrays
 *    are copied during the call.  Every internal buffer is allocated by sem_mesh_setup and
 *    released by sem_destroy.
 *  - All work is enqueued on the context's stream (sem_mesh_desc.stream, a hipStream_t, or the
 *    null stream).  Calls that return values on the host synchronise that stream.
 *  - Every call returns a sem_status and never aborts; no C++ exception crosses the ABI.
 *    sem_last_error() gives the text of the last failure of a context.  SEM_ERR_HIP is sticky:
 *    after it the context only accepts sem_destroy.
 *  - One context per host thread; calls on one context must not overlap.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_ctx sem_ctx;

typedef enum {
  SEM_OK = 0,
  SEM_ERR_ARG = 1,           /* invalid argument or unsupported size                     */
  SEM_ERR_ALLOC = 2,         /* device or host allocation failed                         */
  SEM_ERR_HIP = 3,           /* a HIP runtime call failed (sticky)                       */
  SEM_ERR_NOT_CONVERGED = 4, /* maxit reached; x holds the last iterate                  */
  SEM_ERR_BREAKDOWN = 5,     /* non-finite residual or p.Ap <= 0 in the outer iteration  */
  SEM_ERR_STATE = 6          /* call not valid in the context's current state            */
} sem_status;

/* inner (V-cycle) precision.  SEM_F64 and SEM_F32_GCOL: on 2D levels with equal orders the
 * operator forms its geometric factors in FP64 registers from four values per element column
 * and horizontal node (d, h_x, d_x and the weights, the quantities of Sec. 2.2's sigma
 * derivatives) instead of reading stored factors; SEM_F32 / SEM_F32_GBF16 store the factors in
 * FP32 / BF16 (round to nearest even).  SEM_F32_GCOL is built for 2D meshes; its levels with two
 * orders store FP32 factors. */
enum { SEM_F64 = 0, SEM_F32 = 1, SEM_F32_GBF16 = 2, SEM_F32_GCOL = 3 };
/* smoother on every level above the coarsest.  SEM_SMOOTH_SCHWARZ: the additive Schwarz
 * method of Sec. 5.3, nu_pre / nu_post sweeps of
 * x += W sum_i R_i^T (R_i A R_i^T)^{-1} R_i (b - A x), W = (sum_i R_i^T R_i)^{-1}, over one
 * subdomain per element: the element's nodes widened by sem_mesh_desc.schwarz_overlap node
 * layers across every face (clipped at the domain); 2D and 3D, fine order P <= 8, equal orders
 * along x and sigma.  The inverses of the subdomain blocks are built at set-up (host FP64),
 * rebuilt when the surface moves, and stored per level in the inner precision: E (P_l+1)^4
 * values in 2D without overlap, else E n_max^2 with n_max = prod over the axes of
 * min(nodes along the axis, P_l + 1 + 2 overlap), at most 4096 nodes and 4 GiB of FP64
 * inverses per level (SEM_ERR_ARG beyond). */
enum { SEM_SMOOTH_JACOBI = 0, SEM_SMOOTH_CHEBYSHEV = 1, SEM_SMOOTH_SCHWARZ = 2 };
/* outer iteration */
enum { SEM_OUTER_FPCG = 0, SEM_OUTER_PDC = 1, SEM_OUTER_GMRES = 2 };
/* Dirichlet faces bitmask */
enum { SEM_FACE_TOP = 1 };

#define SEM_MAX_LEVELS 8
#define SEM_MAX_ORDER 12

typedef struct {
  int dim;                     /* 2 or 3                                                    */
  int ne[3];                   /* elements along x, y, z(sigma); ne[1] ignored in 2D        */
  int order;                   /* fine GLL order P, 1..SEM_MAX_ORDER                        */
  int nlevels;                 /* 0: P, ceil(P/2), ..., 1; else level_order[0..nlevels-1]   */
  int level_order[SEM_MAX_LEVELS]; /* strictly decreasing, first = order, last = 1 (with
                                  order_z > 0: the x orders, see level_order_z)               */
  double len[2];               /* horizontal extents L_x, L_y (origin 0)                    */
  const double *h;             /* host: still-water depth at the fine horizontal GLL nodes:
                                  2D (ne[0] P + 1); 3D (ne[0] P + 1) x (ne[1] P + 1), y fastest */
  const double *eta;           /* host: free-surface elevation, same layout as h            */
  unsigned dirichlet_faces;    /* SEM_FACE_TOP (default) or 0 = pure Neumann (apply only)   */
  int inner_prec;              /* SEM_F64 | SEM_F32 | SEM_F32_GBF16 | SEM_F32_GCOL          */
  int smoother;                /* SEM_SMOOTH_*                                               */
  int nu_pre, nu_post;         /* Jacobi and Schwarz sweeps                                 */
  int cheb_degree;             /* Chebyshev degree (pre and post) on the finest level, and on
                                  the coarser levels unless cheb_degree_coarse is set          */
  double jacobi_omega;         /* damping, default 2/3                                      */
  double cheb_lo, cheb_hi;     /* Chebyshev interval as fractions of lambda_hat (0.1, 1.1)  */
  int outer;                   /* SEM_OUTER_FPCG | SEM_OUTER_PDC | SEM_OUTER_GMRES          */
  int maxit;                   /* outer iteration cap                                       */
  int lanczos_steps;           /* steps of the lambda_hat estimate (default 20)             */
  unsigned long long lanczos_seed; /* SplitMix64 seed of the Lanczos start vector           */
  void *stream;                /* hipStream_t or NULL                                        */
  int coarse_dense_max;        /* 3D: below P = 1 the mesh is coarsened in x and y (linear
                                  transfers, same smoother) until a level has at most this many
                                  nodes, which is solved exactly with its dense FP64 inverse
                                  (default 1200).  2D solves P = 1 exactly by block cyclic
                                  reduction and ignores it.                                   */
  int gmres_restart;           /* SEM_OUTER_GMRES: Arnoldi steps per cycle, 1..64
                                  (default 30).  Right-preconditioned GMRES (Sec. 5.4 of the
                                  paper names GMRES beside defect correction): per step one
                                  V-cycle z = B v, one FP64 operator apply and classical
                                  Gram-Schmidt applied twice; x += Z y at the end of a cycle;
                                  sem_solve_info.hist holds the Givens residual estimates of the
                                  steps and, at the end of each cycle, the true residual.      */
  int order_z;                 /* 2D: GLL order along sigma, 1..SEM_MAX_ORDER, when it differs
                                  from `order` (then the order along x); 0 = `order`.  3D: 0 or
                                  equal to `order`.  With different orders the hierarchy is
                                  semi-coarsened (Sec. 5.1): with nlevels = 0 each coarser level
                                  lowers only the larger order, to max(ceil(P/2), the smaller
                                  order), until the two match, then both drop by ceil(P/2)
                                  together down to 1 x 1; a level whose orders differ has no
                                  transfer that changes both directions.  Such levels need
                                  ne[2] (P_x+1) (P_sigma+1) <= 1024, take the Jacobi or Chebyshev
                                  smoother (not Schwarz) and no learned stage.                 */
  int level_order_z[SEM_MAX_LEVELS]; /* with nlevels > 0 and order_z > 0: each level's sigma
                                  order (level_order then holds the x orders); the first equals
                                  order_z, the last 1; from one level to the next neither order
                                  grows and one of them drops, or both drop where both levels
                                  have equal orders.                                          */
  int precond_still_water;     /* 1: every V-cycle level (factors, inverse diagonals, coarse
                                  solve, lambda_hat, the learned stage's geometry) is built from
                                  the still-water geometry eta = 0, the small-amplitude
                                  linearisation that keeps the preconditioner time-constant
                                  (Sec. 5.4); the outer operator, the mass and the faces use the
                                  given eta, and sem_mesh_update_surface never rebuilds the
                                  levels.  0 (default): the levels are built from eta.         */
  int schwarz_overlap;         /* SEM_SMOOTH_SCHWARZ: node layers added to each element's
                                  subdomain across every face, 0..8 (default 0: the element
                                  blocks, neighbouring blocks sharing only face nodes).       */
  int cheb_degree_coarse;      /* Chebyshev degree on every level between the finest and the
                                  coarsest (0, default: cheb_degree).  The one-kernel smoothing
                                  of a 2D coarse level holds its columns plus a halo of one
                                  column per step in a workgroup, so a low degree there keeps
                                  that form when the finest level takes a high one.           */
} sem_mesh_desc;

typedef struct {
  int iters;          /* outer iterations performed                                        */
  int vcycles;        /* V-cycles applied                                                  */
  int learned_skips;  /* learned-stage applications rejected by the judge                  */
  double rel_res;     /* ||b - A x||_2 / ||b||_2 at exit (free and Dirichlet rows)          */
  double ms;          /* wall time of the call                                             */
  int nhist;          /* entries of hist                                                   */
  double hist[512];   /* relative residual after each iteration (hist[0] = initial)         */
  int stage_off_at;   /* learned stage switched off for the rest of the solve after this many
                         iterations, because the judge rejected every application in the
                         last three (0: never)                                              */
} sem_solve_info;

typedef struct {
  int epochs;                /* passes over the training rows (default 30)                  */
  int batch;                 /* rows per Adam step (default 1024)                          */
  float lr;                  /* peak learning rate, cosine decay to 0 (default 1e-3)       */
  float val_frac;            /* trailing fraction of the rows held out (default 0.1)      */
  unsigned long long seed;   /* SplitMix64 seed of the initial weights and shuffles       */
  const void *init;          /* host network blob to start from (NULL: the seeded draw)   */
  size_t init_nbytes;        /* its size in bytes                                         */
} sem_train_cfg;

/* Fill *d with defaults (2D, top Dirichlet, FP64, Chebyshev(3) on [0.1, 1.1] lambda_hat,
 * Jacobi omega 2/3, 2+2 sweeps, FPCG, maxit 500, 20 Lanczos steps, seed 12345, 3D dense
 * coarse level of at most 1200 nodes). */
void sem_mesh_desc_default(sem_mesh_desc *d);

/* Build the level hierarchy, geometric factors, inverse diagonals, lambda_hat estimates and
 * the exact P = 1 coarse factorisation; allocate every buffer.  *out receives the context. */
sem_status sem_mesh_setup(const sem_mesh_desc *desc, sem_ctx **out);

/* Release everything owned by the context (NULL is accepted). */
void sem_destroy(sem_ctx *ctx);

/* Sizes: assembled nodes n_global, free (non-Dirichlet) nodes n_free, element-local nodes
 * n_local = elements (P+1)^dim (2D: elements (P_x+1)(P_sigma+1)).  Any pointer may be NULL. */
sem_status sem_get_sizes(const sem_ctx *ctx, size_t *n_global, size_t *n_free, size_t *n_local);

/* Number of levels of the hierarchy (0 for a NULL context). */
int sem_num_levels(const sem_ctx *ctx);

/* For level l (0 = finest): its order (along x), node count and current lambda_hat. */
sem_status sem_get_level(const sem_ctx *ctx, int level, int *order, size_t *n, double *lambda_hat);

/* For level l (0 = finest): its GLL orders along x and along sigma (they differ on the
 * semi-coarsened levels of a mesh built with order_z != order; 3D: both the order).  Either
 * pointer may be NULL.  SEM_ERR_ARG for a NULL context or a level out of range. */
sem_status sem_get_level_orders(const sem_ctx *ctx, int level, int *order_x, int *order_z);

/* GLL nodes and weights of order P computed by the library (host arrays of P+1). */
sem_status sem_gll(int P, double *nodes, double *weights);

/* Physical coordinates of the nodes of level l (host arrays of that level's node count; y
 * only in 3D, may be NULL in 2D).  Level 0 gives the current surface (after
 * sem_mesh_update_surface); coarser levels the geometry their V-cycle operators were built on. */
sem_status sem_node_coords(const sem_ctx *ctx, int level, double *x, double *y, double *z);

/* Mixed-stage operator (2D).  Inside a Runge-Kutta stage the pressure operator is the
 * divergence at stage k of the gradient taken with stage k-1's sigma transform (Sec. 3.1, eq.
 * poissonp; weak form eq. weak4), read as the bilinear form
 *   a(v, p) = int_{Omega^k} nabla^(k) v . nabla^(k-1) p dOmega^k,
 * nabla^(m) p = (p_x + sigma_x^(m) p_sigma, sigma_z^(m) p_sigma): not symmetric once the two
 * surfaces differ.  eta_prev: host array of stage k-1's surface in the layout of
 * sem_mesh_desc.eta (the current surface is stage k).  The FP64 outer operator
 * (sem_apply_laplacian, sem_assemble_rhs's lifting, the outer iteration) becomes this form until
 * the next sem_mesh_update_surface or a call with eta_prev = NULL; the V-cycle stays the
 * (time-constant) preconditioner.  sem_poisson_solve then needs SEM_OUTER_GMRES or
 * SEM_OUTER_PDC (SEM_ERR_STATE with FPCG).  SEM_ERR_ARG in 3D or if h + eta_prev <= 0. */
sem_status sem_mesh_mixed_stage(sem_ctx *ctx, const double *eta_prev);

/* ---- the stage loop (Sec. 3) around the solve ----------------------------------------------
 * The paper advances its model with the five-stage fourth-order low-storage Runge-Kutta scheme
 *   K^k = alpha_k K^(k-1) + dt f(y^(k-1), t_n + c_k dt),  y^(k) = y^(k-1) + beta_k K^k,
 * solving a Poisson problem on the mesh of every stage's surface with a time-constant
 * preconditioner (Sec. 5.4; sem_mesh_desc.precond_still_water).  Its velocity-dependent
 * right-hand side is outside this library; the stage loop here is driven by the linear
 * free-surface potential-flow model on the same meshes, state y = (eta, Phi) at the surface
 * nodes (2 ns values, ns = ne[0] P + 1 in 2D, (ne[0] P + 1)(ne[1] P + 1) in 3D, each half in the
 * layout of sem_mesh_desc.eta):  -lap phi = 0 with phi = Phi on the surface and zero normal
 * derivative on walls and bottom, d eta/dt = d phi/dz at the surface, d Phi/dt = -g eta. */

/* The scheme's coefficients alpha, beta, c (five each; the published fourth-order 2N-storage
 * solution of Carpenter and Kennedy, 1994, which the paper cites without printing). */
void sem_lserk_coefficients(double *alpha, double *beta, double *c);

/* Stage update k (0..4) on device arrays of n values: K = alpha_k K + dt F; y += beta_k K,
 * on the context's stream.  SEM_ERR_ARG for a bad stage or null pointers. */
sem_status sem_lserk_update(sem_ctx *ctx, int stage, double dt, const double *F, double *K,
                            double *y, size_t n);

/* w = d phi / dz at the surface nodes of the current fine mesh: (1/d) d phi / d sigma
 * (Sec. 2.2, sigma_z = 1/d) from the top element's nodal values with the GLL differentiation
 * matrix.  phi: device, the fine level's n_global values; w: device, ns values. */
sem_status sem_surface_dz(sem_ctx *ctx, const double *phi, double *w);

/* The model's right-hand side F = f(y) (device arrays of 2 ns values): the mesh follows eta
 * (sem_mesh_update_surface without refreshing the preconditioner; eta is copied to the host
 * for it), phi solves the Dirichlet problem with Phi on the surface (sem_poisson_solve to tol,
 * warm-started from phi, which is a device array of n_global values updated in place), then
 * F = (d phi / dz at the surface, -g eta).  info (may be NULL) receives the solve's record. */
sem_status sem_wave_rhs(sem_ctx *ctx, const double *y, double *F, double *phi, double g,
                        double tol, sem_solve_info *info);

/* One step of the scheme for the model: five sem_wave_rhs / sem_lserk_update pairs on y (2 ns
 * device values, advanced in place) with the stage vector K (2 ns device values, overwritten).
 * iters (may be NULL): the five solves' iteration counts. */
sem_status sem_wave_step(sem_ctx *ctx, double *y, double *K, double *phi, double dt, double g,
                         double tol, int *iters);

/* New free surface for a time series.  The sigma transform follows eta (Sec. 2.2, eq. sigtrans),
 * so the operator's geometric factors change with it; the paper keeps the multigrid
 * preconditioner time-constant (Sec. 5.4).  eta: host array in the layout of sem_mesh_desc.eta
 * (copied).  The FP64 outer operator (sem_apply_laplacian, the outer iteration of
 * sem_poisson_solve), the lumped mass and the wall-face weights (sem_assemble_rhs) are rebuilt
 * for the new surface (in 3D on the device).  refresh_precond = 0 keeps every V-cycle level as
 * it is (frozen preconditioner; FPCG converges to the new operator's solution); 1 rebuilds
 * every level too (factors, inverse diagonals, coarse solve, lambda_hat estimates and the
 * learned stage's geometry; host work of the order of the set-up).  Errors: SEM_ERR_ARG if eta is
 * NULL or h + eta <= 0 anywhere (the context is left unchanged). */
sem_status sem_mesh_update_surface(sem_ctx *ctx, const double *eta, int refresh_precond);

/* y = A x on the fine level in FP64: the assembled GLL stiffness (sum of element matrices,
 * Sec. 4.2 eq. globallocal) of the symmetric sigma-Laplacian, restricted to free rows and
 * columns, with identity rows on Dirichlet nodes (pure Neumann if dirichlet_faces = 0).
 * x, y: device, n_global doubles, must not alias. */
sem_status sem_apply_laplacian(sem_ctx *ctx, const double *x, double *y);

/* The same operator on level l in the context's inner precision (x is rounded to it, the
 * result widened to FP64).  Test hook for the inner-precision apply. */
sem_status sem_apply_level(sem_ctx *ctx, int level, const double *x, double *y);

/* z = B r: one p-multigrid V-cycle (Sec. 5) from a zero initial guess in the inner precision:
 * pre-smoothing on every level above the coarsest, residual, restriction R = P^T (Sec. 5.2),
 * exact FP64 solve on P = 1, prolongation by interpolation, post-smoothing.  r, z: device,
 * n_global doubles; r must be zero on Dirichlet rows (z is then zero there). */
sem_status sem_pmg_vcycle(sem_ctx *ctx, const double *r, double *z);

/* Solve A x = rhs to ||rhs - A x||_2 <= tol ||rhs||_2 with the outer loop chosen at setup
 * (flexible CG or defect correction, each preconditioned by one V-cycle), all outer vectors,
 * the outer operator and inner products in FP64.  rhs must hold g_D on Dirichlet rows (see
 * sem_assemble_rhs).  x: initial guess on entry, solution on exit.  rhs and x are device
 * n_global doubles and must not alias.  info may be NULL.  Returns SEM_ERR_NOT_CONVERGED
 * (x = last iterate) or SEM_ERR_BREAKDOWN (x = last finite iterate) on failure. */
sem_status sem_poisson_solve(sem_ctx *ctx, const double *rhs, double *x, double tol,
                             sem_solve_info *info);

/* rhs = M f + B g_N - A_fD g_D on free rows, rhs = g_D on Dirichlet rows (Sec. 4.2 eq.
 * fsemidiscrete with the lumped GLL mass M and GLL face quadrature B).
 *   f   : device, n_global doubles (nodal source values) or NULL for f = 0
 *   gN  : device, per-face nodal values of n . grad p, packed faces in this order:
 *         2D: x = 0 wall (Nz P + 1), x = L_x wall (Nz P + 1), bottom (Nx P + 1);
 *         3D: x = 0, x = L_x [(Ny P + 1)(Nz P + 1) each, z fastest], y = 0, y = L_y
 *         [(Nx P + 1)(Nz P + 1) each], bottom [(Nx P + 1)(Ny P + 1), y fastest]; or NULL
 *   gD  : device, free-surface values (one per top node, in global order) or NULL for 0
 *   rhs : device, n_global doubles (output). */
sem_status sem_assemble_rhs(sem_ctx *ctx, const double *f, const double *gN, const double *gD,
                            double *rhs);

/* Override lambda_hat (largest eigenvalue estimate of D^{-1} A) of level l (l above the
 * coarsest).  Parity tests inject the reference value. */
sem_status sem_set_smoother_bounds(sem_ctx *ctx, int level, double lambda_hat);

/* Test hooks for single steps of the V-cycle, FP64 device vectors of the level sizes:
 *   sem_restrict     rc = P^T (b - A x) on level l -> l+1, coarse Dirichlet rows zeroed
 *                    (x = NULL means x = 0, i.e. rc = P^T b)
 *   sem_prolong_add  xf += P ec, level l+1 -> l
 *   sem_smooth       x <- smoother(b, x) on level l (pre = 1: from x = 0, x is output only)
 *   sem_coarse_solve x = A_1^{-1} b on the coarsest level (exact, FP64). */
sem_status sem_restrict(sem_ctx *ctx, int level, const double *b, const double *x, double *rc);
sem_status sem_prolong_add(sem_ctx *ctx, int level, const double *ec, double *xf);
sem_status sem_smooth(sem_ctx *ctx, int level, int pre, const double *b, double *x);
sem_status sem_coarse_solve(sem_ctx *ctx, const double *b, double *x);

/* Benchmark hook: launch a kernel of level l reps times on the context's stream, bracketed by
 * HIP events recorded on that stream, and return the average time per launch in *ms_avg.
 * kind 0: the level's inner-precision operator; kind 1: the fine-level FP64 operator of the
 * outer loop (level 0 only); kind 2: the level's fused smoother step (operator and Chebyshev
 * update in one kernel, 2D levels where it fits, else SEM_ERR_ARG), with d read and written.
 * flush = 0 times back-to-back launches on the same buffers (whose data then stays in the
 * 256 MB Infinity Cache when it fits); flush = 1 overwrites a 512 MiB device buffer before every
 * launch (cold caches) and times each launch separately (event overhead included); flush = 2
 * makes R copies of every buffer the kernel reads or writes (R of them exceed 768 MiB, R <= 64;
 * allocated for the call and freed before it returns) and times at least 2R back-to-back
 * launches that take the copies in turn, so each launch streams its data from HBM.  Inputs are
 * the level's own work vectors, which are overwritten; results are discarded.  Synchronises the
 * stream. */
sem_status sem_time_operator(sem_ctx *ctx, int level, int kind, int reps, int flush,
                             double *ms_avg);

/* Benchmark hook: one sem_poisson_solve (same arguments and result) run with every launch
 * issued directly instead of replayed from graphs, and *bytes = the sum over its launches of
 * each kernel's algorithmic bytes (every array it reads or writes counted once at its logical
 * size, factors in their storage precision, block-reduction factors once per application; no
 * re-reads, halos or scratch).  *iters (may be NULL): outer iterations; *launches (may be
 * NULL): kernels counted.  Returns the solve's status.  Not for concurrent use from several
 * host threads (the tally is per process). */
sem_status sem_solve_bytes(sem_ctx *ctx, const double *rhs, double *x, double tol, double *bytes,
                           int *iters, long *launches);

/* Algorithmic bytes of one launch of sem_time_operator's kernel (every vector read or written
 * once, every geometric factor read once): kind 0, 1: x read, y written; kind 2: x, b, dinv, d
 * read, x, d written; plus the factors in their storage precision. */
sem_status sem_operator_bytes(const sem_ctx *ctx, int level, int kind, double *bytes);

/* Test hook: launch shape of level l's 2D kernels.  *cols_per_block: element columns owned by
 * one workgroup of the fused smoother step in the level's precision (0: the level has no fused
 * step: 3D, the coarsest level, or columns too tall for one workgroup); *coarse_w: owned columns
 * per workgroup of the one-kernel pre-smoothing of a coarse level (level >= 1; 0: per-step
 * kernels).  Either pointer may be NULL.  SEM_ERR_ARG for a NULL context or a bad level. */
sem_status sem_launch_shape(const sem_ctx *ctx, int level, int *cols_per_block, int *coarse_w);

/* ---- learned smoothing stage (not in the paper; an addition beside the method) -------------
 * An element-local MLP maps each element's restricted residual r_e = R_e r (R_e: the element
 * restriction, the R_i of the paper's Schwarz smoother, Sec. 5.3) plus its geometric factors to a
 * correction.  Features per element (n = (P+1)^2 nodes, local order i*(P+1)+j):
 *   [r_e / s_e, G_rr / g_e, G_rs / g_e, G_ss / g_e, m_e / mean(m_e)],  s_e = ||r_e||_2,
 *   g_e = mean over the element of (G_rr + G_ss);
 * network 5n -> 128 -> 128 -> n, exact-erf GELU on the hidden layers, BF16 operands with FP32
 * accumulation on the matrix cores; correction c = W sum_e R_e^T (s_e / a_e) y_e with a_e the
 * mean diagonal of the element matrix and W the averaging weight of Sec. 5.3, zero on the
 * surface.  In the V-cycle the stage runs on the finest level after pre-smoothing: q = A c,
 * alpha = c.r / c.q (energy-optimal), accepted if alpha > 0 and finite (x += alpha c: the A-norm
 * of the error never grows), otherwise skipped and counted in sem_solve_info.learned_skips; after
 * three outer iterations in a row in which every application was rejected, sem_poisson_solve
 * switches the stage off for the rest of that solve (sem_solve_info.stage_off_at).  3D meshes
 * (hexahedra, P <= 6): the same stage with 7n inputs (the residual, the factor fields G_rr, G_tt,
 * G_rs, G_ts, G_ss over g_e = mean(G_rr + G_tt + G_ss), the mass), n = (P+1)^3.  Training pairs: target
 * t_e = (a_e / s_e) R_e e for the error e; loss = mean squared error; Adam.
 * Network blob: 64-byte header ("SEMN", version 1, sizes, seed, losses) followed by FP32
 * W1 [nin x 128], b1, W2 [128 x 128], b2, W3 [128 x nout], b3, row-major. */

/* Bytes of a network blob with nin inputs and nout outputs. */
size_t sem_mlp_blob_size(int nin, int nout);

/* Training features of the fine level (2D, P <= 8, X [E x 5n]; 3D, P <= 6, X [E x 7n]): for an
 * assembled residual r (device FP64, n_global) write X and, if T is given, targets T [E x n]
 * (device FP32, row-major;
 * E = elements): with an error e, t_e = (a_e / s_e) R_e e; with e = NULL, the element-block solve
 * t_e = (a_e / s_e) (R_e A R_e^T)^{-1} R_e r (the local solve of the Schwarz smoother, Sec. 5.3;
 * meshes up to 4096 elements in 2D, 1024 in 3D). */
sem_status sem_learned_features(sem_ctx *ctx, const double *r, const double *e, float *X,
                                float *T);

/* Training pairs of the learned stage from this context's own p-multigrid (2D, fine order
 * P <= 8, at most 4096 elements, FP64 context recommended).  For cycles >= 1: defect-correction
 * cycles x <- x + B (b - A x) from x = 0 on the right-hand side b (device FP64, n_global, zero
 * on the surface rows); at each cycle, at the point where the stage acts (the fine level after
 * pre-smoothing of the cycle's residual r from zero: r_pre = r - A S(r)), rows of features
 * X [rows x 5n] and element-block targets T [rows x n] (the features and targets of
 * sem_learned_features with e = NULL) are written for `per` elements drawn without
 * replacement by a SplitMix64-driven Fisher-Yates prefix (seed, draws counted through the call;
 * per = 0: every element in order).  cycles = 0: one set of rows for b itself as the residual.
 * The stage does not act in these cycles.  X, T: device FP32 with room for
 * max(cycles, 1) * (per or E) rows; *rows receives the count written (may be NULL). */
sem_status sem_learned_harvest(sem_ctx *ctx, const double *b, int cycles, int per,
                               unsigned long long seed, float *X, float *T, size_t *rows);

/* Train the learned stage's network for this context's fine level (nin = 5n, nout = n) on
 * device rows X [n x nin], T [n x nout] (FP32; e.g. from sem_learned_harvest) with the
 * library's BF16 MFMA forward/backward kernels (FP32 accumulation, FP32 master weights), Adam
 * (beta 0.9 / 0.999, eps 1e-8) and a cosine learning rate from cfg->lr to 0 over all steps
 * (cfg NULL: defaults).  blob: host buffer of *nbytes bytes (at least sem_mlp_blob_size(5n, n));
 * *nbytes receives the blob's size.  The trained network is also loaded into the context, with
 * the stage's placement as it was (off if no network was loaded before). */
sem_status sem_learned_train(sem_ctx *ctx, const float *X, const float *T, int n,
                             const sem_train_cfg *cfg, void *blob, size_t *nbytes);

/* The same training without a context, for any nin, nout: device rows X [n x nin], T [n x nout]
 * (FP32).  blob: host buffer of sem_mlp_blob_size(nin, nout) bytes (output).  losses: host
 * array of 2*epochs floats (training loss of the last batch, validation loss) or NULL.  Errors
 * are reported through sem_last_error(NULL). */
sem_status sem_mlp_train(const float *X, const float *T, int n, int nin, int nout,
                         const sem_train_cfg *cfg, void *blob, size_t nbytes, float *losses);

/* Test hooks of the training kernels: batched forward Y [n x nout] of device rows X, and the
 * loss and parameter gradients (host array packed like the blob parameters) of device rows
 * X, T.  blob: host. */
sem_status sem_mlp_forward(const void *blob, size_t nbytes, const float *X, int n, float *Y);
sem_status sem_mlp_gradients(const void *blob, size_t nbytes, const float *X, const float *T,
                             int n, float *grads, float *loss);

/* sem_mlp_forward for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same kernels and the same results, with
 * the network and the activations of one 256-row chunk held in a fixed device array of the
 * library (about 1.2 MB, one copy per GPU, kept until the process ends) instead of buffers
 * allocated per call.  The call allocates nothing and frees nothing; it runs on the null stream
 * and synchronises it.  Limits: nin <= 416 and nout <= 96 (SEM_ERR_ARG beyond), any n >= 1.
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU race. */
sem_status sem_mlp_forward_noalloc(const void *blob, size_t nbytes, const float *X, int n,
                                   float *Y);

/* Load a network blob (host) into the context (nin = 5n in 2D, 7n in 3D, nout = n, the nodes of
 * a fine-level element; 2D P <= 8, 3D P <= 6) and
 * set where the stage acts: enable = 0 off, bit 0 (1) after the finest pre-smoothing, bit 1 (2)
 * before the finest post-smoothing (3 = both, keeping the V-cycle close to symmetric for the
 * flexible-CG outer loop); sem_learned_enable changes it for a loaded network. */
sem_status sem_learned_load(sem_ctx *ctx, const void *blob, size_t nbytes, int enable);
sem_status sem_learned_enable(sem_ctx *ctx, int enable);

/* Test hook: one learned stage on the fine level for b, x (device FP64, x updated in place);
 * *accepted = 1 if the step was taken. */
sem_status sem_learned_stage(sem_ctx *ctx, const double *b, double *x, int *accepted);

/* Number of learned-stage applications the judge rejected since the last reset (solves reset
 * it on entry; sem_pmg_vcycle and sem_learned_stage do not).  reset != 0 sets it to zero after
 * reading.  SEM_ERR_STATE if no network was ever loaded. */
sem_status sem_learned_skips(sem_ctx *ctx, int *skips, int reset);

/* The plain smoother as the judge of the learned stage, by residual reduction per cycle and
 * per unit of time: for A x = rhs (rhs: device FP64, n_global, as for sem_poisson_solve) the
 * call runs defect-correction cycles x += B(rhs - A x) from x = 0, with the stage off and then
 * on (its placement from sem_learned_load / sem_learned_enable, after pre-smoothing if it is
 * off), one cycle untimed and `cycles` timed (1..100) each, every cycle one captured HIP graph
 * (launched directly under SEM_NO_GRAPH=1, as the solves are), timed with HIP events on the
 * library stream.  rho = (||r_end|| / ||r_start||)^(1/cycles)
 * over the timed cycles, ms the time per cycle.  The stage is left enabled iff it reduces the
 * residual faster per unit of time (rho_learned < 1 and ln(rho_learned) / ms_learned <
 * ln(rho_plain) / ms_plain), else disabled (as sem_learned_enable(ctx, 0)); the rejection
 * counter is reset.  out (may be NULL) receives both measurements and the decision.
 * SEM_ERR_STATE without a loaded network. */
typedef struct {
  double rho_plain, rho_learned;   /* residual reduction per cycle, stage off / on       */
  double ms_plain, ms_learned;     /* milliseconds per cycle, stage off / on             */
  int enabled;                     /* 1: the stage stays on                              */
} sem_judge_result;
sem_status sem_learned_judge(sem_ctx *ctx, const double *rhs, int cycles, sem_judge_result *out);

/* Text of the last error on this context ("" if none).  Valid until the next call. */
const char *sem_last_error(const sem_ctx *ctx);

/* Name of a status code. */
const char *sem_status_string(sem_status s);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
