/*
 * eqs.h - C ABI of the MI355X (gfx950) explicit-RKC library for nonlinear
 * electro-quasistatic (EQS) fields.
 *
 * Method: C. Richter, S. Schoeps, M. Clemens, "GPU Accelerated Explicit Time
 * Integration Methods for Electro-Quasistatic Fields" (arXiv 1612.09447).
 *   Sec. II, eq. (1): div(kappa(|grad phi|) grad phi) + div(eps grad dphi/dt) = 0.
 *   Sec. II, eq. (2): after P1 finite elements, M dx/dt + K(x)x = b, with M the
 *     constant permittivity Laplacian, K(x) the field-dependent conductivity
 *     matrix and b the inhomogeneous Dirichlet contribution.
 *   Sec. II: explicit Runge-Kutta-Chebyshev (RKC, its ref. [9]) time stepping,
 *     where every stage needs one solve with the constant M (a multiple
 *     right-hand-side problem whose preconditioner is built once).
 *   Sec. III: K(x)x is formed element by element and added straight into the
 *     right-hand side; the matrix K(x) is never assembled.
 *   Sec. II/V: M is solved by conjugate gradients with an algebraic multigrid
 *     preconditioner.
 *
 * Conventions for every call:
 *   - Return value: EQS_OK (0) or a negative EQS_ERR_* code; the thread-local
 *     message of the last failure is eqs_last_error(). No C++ exception ever
 *     crosses this interface.
 *   - Host arrays passed to eqs_set_* are copied; the caller keeps ownership
 *     and may free them after the call returns.
 *   - Device pointers (suffix _dev) must be device memory on the context's
 *     device, 8-byte aligned, and are only borrowed for the duration of the
 *     call. All device work is enqueued on the context's stream; calls return
 *     after that work has completed (the library synchronises its stream), so
 *     results are ready for any stream afterwards.
 *   - Node ids are 0-based int32. "Free" nodes are the nodes not listed in
 *     eqs_set_dirichlet; vectors over free nodes (length n_free) list them in
 *     increasing node id. Vectors over all nodes (length n_nodes) are in node
 *     id order.
 *   - Units are SI: metres, volts, seconds, S/m; eps = eps0 * eps_r with
 *     eps0 = 8.8541878128e-12 F/m.
 *   - A context is not thread-safe; separate contexts are independent.
 */
#ifndef EQS_H
#define EQS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define EQS_OK 0
#define EQS_ERR_INVALID_ARG (-1)   /* bad pointer, size, id, or degenerate tet */
#define EQS_ERR_STATE (-2)         /* call out of order (see eqs_build_preconditioner) */
#define EQS_ERR_HIP (-3)           /* HIP runtime error */
#define EQS_ERR_NOT_CONVERGED (-4) /* maxit reached; results and stats still written */
#define EQS_ERR_BREAKDOWN (-5)     /* CG breakdown: p.Mp <= 0 or non-finite scalar */
#define EQS_ERR_NONFINITE (-6)     /* NaN/Inf in an input */
#define EQS_ERR_ALLOC (-7)         /* device or host allocation failed */

#define EQS_MAX_DRIVES 65536 /* distinct drive functions per context */

enum { EQS_PREC_FP64 = 0, EQS_PREC_FP32 = 1 };

typedef struct eqs_ctx eqs_ctx;

/* Material law (Sec. I and eq. (1)): permittivity eps0*eps_r; conductivity
 * kappa0 * (1 + (|E|/e_s)^alpha) if nonlinear != 0 (a microvaristor-type
 * power law switching near the field e_s), else the constant kappa0.
 * Requires eps_r > 0, kappa0 >= 0, and for nonlinear materials e_s > 0,
 * alpha >= 0. */
typedef struct eqs_material {
    double eps_r;
    double kappa0;
    double e_s;
    double alpha;
    int32_t nonlinear;
    int32_t reserved; /* set to 0 */
} eqs_material;

/* Dirichlet drive g(t) = amp * sin(2 pi freq t + phase) (amp = 0: ground;
 * freq = 0, phase = pi/2: constant amp). Its time derivative enters b of
 * eq. (2). */
typedef struct eqs_drive {
    double amp;
    double freq;
    double phase;
} eqs_drive;

/* Smoothed-aggregation AMG parameters for the preconditioner of M (the
 * paper's solver is AMG-preconditioned CG, Sec. I and Sec. V; the algebraic
 * multigrid variant is this library's choice). Zero-initialised fields take
 * the defaults in brackets. */
typedef struct eqs_amg_params {
    int32_t precision;  /* EQS_PREC_FP64 or EQS_PREC_FP32 storage and V-cycle [FP64] */
    int32_t coarse_max; /* coarsen until at most this many unknowns, <= 4096 [512] */
    int32_t max_levels; /* including the coarsest, 2..16 [12] */
    int32_t flexible;   /* CG beta: 1 Polak-Ribiere (flexible), 2 Fletcher-Reeves; 0 = PR with FP32, FR with FP64 */
    double theta;       /* strength threshold |a_ij| >= theta sqrt(a_ii a_jj) at the finest level,
                           halved per level [0.02] */
    double jacobi_weight; /* damped-Jacobi weight times 1/rho(D^-1 A) [3/2] */
    double smooth_weight; /* prolongator-smoothing weight times 1/rho(D^-1 A) [4/3] */
} eqs_amg_params;

typedef struct eqs_solve_stats {
    int32_t iters;  /* CG iterations */
    int32_t status; /* EQS_OK, EQS_ERR_NOT_CONVERGED or EQS_ERR_BREAKDOWN */
    double relres;  /* true |rhs - M y| / |rhs| at exit (0 if rhs = 0) */
} eqs_solve_stats;

typedef struct eqs_step_stats {
    int32_t stages;          /* s */
    int32_t total_iters;     /* CG iterations summed over the stages */
    int32_t max_iters;       /* largest per-stage count */
    int32_t min_iters;       /* smallest per-stage count */
    int32_t not_converged;   /* stages whose solve hit maxit */
    int32_t guess_used;      /* stages whose CG started from the estimator's vector */
    int32_t guess_fallbacks; /* stages where the guard kept the previous solution instead */
    int32_t reserved;
    double max_relres;       /* largest per-stage true relative residual */
    double train_loss;       /* last minibatch loss of the start-vector network (0 if none) */
} eqs_step_stats;

typedef struct eqs_info {
    int64_t n_nodes;
    int64_t n_tets;
    int64_t n_free;
    int64_t nnz_M;        /* nonzeros of M restricted to the free nodes */
    int32_t n_levels;     /* AMG levels including the coarsest (0 before build) */
    int32_t precision;
    int64_t level_rows[16];
    int64_t level_nnz[16];   /* nonzeros of the level operator A_l */
    int64_t level_p_nnz[16]; /* nonzeros of the prolongation P_l (level l+1 -> l; 0 on the coarsest) */
    int64_t level_r_nnz[16]; /* nonzeros of the restriction applied at level l (R_l = P_l^T, or
                                R_l (I - A_l w D_l^-1) where the pre-smoother is folded in) */
    int64_t device_bytes;    /* device memory the library allocated itself for the context */
    int64_t workspace_bytes; /* size of the caller's workspace (0: none attached) */
    int64_t workspace_used;  /* bytes of it the context's buffers occupy */
} eqs_info;

/* Create a context on HIP device `device` whose work goes to `hip_stream`
 * (a hipStream_t; NULL = the null stream). *out receives the context. */
int eqs_create(eqs_ctx **out, int device, void *hip_stream);

/* Release the context and all device memory it holds. NULL is accepted. */
int eqs_destroy(eqs_ctx *ctx);

/* Tetrahedral P1 mesh (the "FEM data" handed to the GPU, Sec. III).
 * xyz: n_nodes x 3 doubles (x, y, z per node); tets: n_tets x 4 node ids.
 * Every tet needs a nonzero volume (either orientation); a flat tet gives
 * EQS_ERR_INVALID_ARG. Resets materials, Dirichlet data and the preconditioner. */
int eqs_set_mesh(eqs_ctx *ctx, int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets);

/* The same with second-order (10-node) tetrahedra (Sec. III's P2 elements;
 * Sec. V's second-order model): tets is n_tets x 10, the four vertices, then
 * the midpoints of the edges (0,1), (0,2), (0,3), (1,2), (1,3), (2,3). Elements
 * are straight-sided: only the vertex coordinates enter the geometry. M is
 * integrated exactly (4-point rule of degree 2) and K(x)x takes kappa(|E|) at
 * those four points, where the field is linear on the element.
 * eqs_rkc_adaptive and batches are built for 4-node tets only. */
int eqs_set_mesh_p2(eqs_ctx *ctx, int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets);

/* Material table (n_mat entries) and the material id of every tet
 * (tet_mat[n_tets], 0 <= id < n_mat <= 65535): the "nonlinear material
 * parameters" of Sec. III. Invalidates the preconditioner. */
int eqs_set_materials(eqs_ctx *ctx, int32_t n_mat, const eqs_material *mats, const int32_t *tet_mat);

/* Dirichlet nodes and their drives (eq. (1) is well posed with Dirichlet
 * data, Sec. II): node nodes[k] follows drives[drive_id[k]]. Nodes must be
 * distinct; 1 <= n_drive <= EQS_MAX_DRIVES; at least one node must stay
 * free. All other boundary parts are natural (zero normal current).
 * Invalidates the preconditioner. */
int eqs_set_dirichlet(eqs_ctx *ctx, int64_t n_d, const int32_t *nodes, const int32_t *drive_id,
                      int32_t n_drive, const eqs_drive *drives);

/* Checkpoint and resume of a run (the state the RKC steps of Sec. II carry
 * from one step to the next inside the context). Between steps, the state of
 * a built context - the last stage solution F (the next step's first start
 * vector, Sec. IV) and its M-product, the start-vector window with its
 * reduced matrices, the network's weights and Adam moments, its replay buffer
 * and sampling counter - is written to a host buffer the caller owns;
 * eqs_state_load restores it into a context built from the same mesh,
 * materials, Dirichlet data, instances and precision and given the same
 * eqs_set_guess settings, so that the run continues as if it had not stopped
 * (bit for bit with eqs_set_deterministic). The potentials themselves are the
 * caller's (x of eqs_rkc_step). eqs_state_size gives the bytes a save needs
 * (at 2.1 M free DOF: 34 MB, plus 16 window vectors of 17 MB each with an
 * estimator start vector); save fails with EQS_ERR_INVALID_ARG if `bytes` is
 * smaller; load fails with EQS_ERR_INVALID_ARG if the buffer is not a
 * checkpoint of such a context (after a failed load the run state may be
 * partly overwritten: load a valid checkpoint, or call eqs_set_guess, before
 * the next step). All three synchronise the context's streams. */
int eqs_state_size(eqs_ctx *ctx, int64_t *bytes);
int eqs_state_save(eqs_ctx *ctx, void *host_buf, int64_t bytes);
int eqs_state_load(eqs_ctx *ctx, const void *host_buf, int64_t bytes);

/* Deterministic element pass (the fused K(x)x of Sec. III): with on = 1 the
 * element contributions are summed in an order fixed at set-up (each tet
 * writes its four values to slots of its block; every block node sums its
 * slots in order; every node sums its blocks' partials in block order)
 * instead of by floating-point atomics, so K(x)x, the stage right-hand side
 * and therefore whole RKC trajectories are the same bit for bit from run to
 * run (across separately built contexts when they use the same operator
 * layouts: EQS_TUNE_FILE or EQS_AUTOTUNE=0 fix those). It costs about 160 MB of lists and partials at 12.6 M tets and extra
 * memory traffic per pass. First-order tets only. Must be set before
 * eqs_build_preconditioner (EQS_ERR_STATE afterwards if it would change);
 * [0]. */
int eqs_set_deterministic(eqs_ctx *ctx, int32_t on);

/* Launch granularity of the CG solves (the solve is Sec. II's M-solve; the
 * grouping is this library's choice): every launch replays one captured HIP
 * graph of `iters` CG iterations, 1..EQS_MAX_GRAPH_ITERS [1]. Iterations that
 * a launch holds past convergence change nothing: their preconditioner cycle
 * runs (its kernels do not test the stop flag, which would cost every one of
 * them a wait), and their SpMV, update and scalar kernels return at entry.
 * So a large value gives a graph spanning the whole solve at the price of
 * those cycles, a small one lets the host stop at convergence. Results do not
 * depend on it. Takes effect at the next solve; EQS_ERR_INVALID_ARG outside
 * the range. */
#define EQS_MAX_GRAPH_ITERS 256
int eqs_set_graph_iters(eqs_ctx *ctx, int32_t iters);

/* Assemble M on the free nodes (eq. (2)), build the AMG hierarchy once for
 * all stages and steps (Sec. II: the constant M makes the solves a multiple
 * right-hand-side problem), and upload mesh, materials and hierarchy to the
 * device. Needs mesh, materials and Dirichlet data, else EQS_ERR_STATE.
 * p may be NULL for the defaults. */
int eqs_build_preconditioner(eqs_ctx *ctx, const eqs_amg_params *p);

/* Sizes and hierarchy statistics. */
int eqs_get_info(const eqs_ctx *ctx, eqs_info *info);

/* ---- device memory from the caller ------------------------------------
 * Every device buffer of a context (mesh, M, the AMG hierarchy, the CG and
 * RKC vectors, the start-vector window and network) is one of a set of
 * 256-byte-aligned blocks; the library allocates them itself unless the
 * caller supplies one workspace that holds them all, so that a framework's
 * allocator (PyTorch's) can own all device memory.
 *
 * eqs_query: after eqs_build_preconditioner, *n_free (may be NULL) receives
 * the number of free nodes and *ws_bytes (may be NULL) the workspace size the
 * context needs for its present configuration: its buffers plus those the
 * start-vector settings of eqs_set_guess will allocate on their first stage
 * (query after eqs_set_guess to include them). EQS_ERR_STATE before the build.
 *
 * eqs_set_workspace: dev (device memory on the context's device, 256-byte
 * aligned, `bytes` long, not freed by the caller while attached) becomes the
 * context's device memory: a built context's buffers move into it (device
 * copies, on the context's stream) and the memory the library had allocated
 * is released, so eqs_get_info then reports device_bytes = 0; buffers the
 * context allocates later (the start-vector window on its first stage, a
 * rebuild) come from the workspace's free space, and EQS_ERR_ALLOC reports
 * a workspace that cannot hold them (a rebuild also needs room for the
 * trial layouts the set-up times). bytes below eqs_query's size gives
 * EQS_ERR_INVALID_ARG and leaves the context as it was. dev = NULL moves the
 * buffers back into memory the library allocates and detaches the workspace.
 * The workspace stays attached until eqs_destroy, another eqs_set_workspace,
 * or eqs_set_workspace(ctx, NULL, 0). Calling eqs_set_workspace before the
 * build makes the build itself allocate from it. */
int eqs_query(const eqs_ctx *ctx, int64_t *n_free, int64_t *ws_bytes);
int eqs_set_workspace(eqs_ctx *ctx, void *dev, int64_t bytes);

/* y = K(x_bar) x_bar on all nodes (Sec. III, element-by-element product),
 * where x_bar equals x_dev on free nodes and g(t) on Dirichlet nodes
 * (the Dirichlet entries of x_dev are ignored). x_dev, y_dev: n_nodes
 * doubles, may not alias. */
int eqs_apply_K(eqs_ctx *ctx, double t, const double *x_dev, double *y_dev);

/* Stage right-hand side r = b(t) - [K(x_bar) x_bar]_free with
 * b(t) = -M_{free,D} g'(t) (eq. (2) with the Dirichlet nodes D eliminated)
 * and x_bar = (y_free_dev, g(t)). Both vectors have n_free doubles. */
int eqs_stage_rhs(eqs_ctx *ctx, double t, const double *y_free_dev, double *r_dev);

/* y = M_free x (the constant matrix of eq. (2) on the free nodes). */
int eqs_apply_M(eqs_ctx *ctx, const double *x_dev, double *y_dev);

/* z = B r: one AMG V-cycle applied to r (the preconditioner built by
 * eqs_build_preconditioner; linear and symmetric positive definite). */
int eqs_apply_preconditioner(eqs_ctx *ctx, const double *r_dev, double *z_dev);

/* Solve M_free y = rhs by AMG-preconditioned CG (Sec. II, Sec. V) until the
 * true relative residual |rhs - M y| / |rhs| <= rtol. y_dev holds the start
 * vector on entry (Sec. IV: a good start vector cuts iterations; an exact one
 * needs none) and the solution on exit. Returns EQS_ERR_NOT_CONVERGED after
 * maxit iterations (y and stats still written) or EQS_ERR_BREAKDOWN.
 * st may be NULL. */
int eqs_solve_M(eqs_ctx *ctx, const double *rhs_dev, double *y_dev, double rtol, int32_t maxit,
                eqs_solve_stats *st);

/* One RKC step (Sec. II, its ref. [9]: s stages, second order, damping 2/13)
 * from time t to t + dt for M dx/dt + K(x)x = b. x_dev (n_nodes doubles) holds
 * x(t) on entry (Dirichlet entries ignored) and x(t + dt) on exit, with the
 * Dirichlet entries set to g(t + dt). Every stage j evaluates
 * F_j = M^{-1}(b(t + c_j dt) - K(x_bar_j) x_bar_j) with one fused element pass
 * and one preconditioned CG solve to rtol, started from the previous stage's
 * F. Requires 2 <= s <= 256. Returns EQS_ERR_NOT_CONVERGED if any stage's
 * solve hit maxit (the step is still completed); st may be NULL. */
int eqs_rkc_step(eqs_ctx *ctx, double t, double dt, int32_t s, double *x_dev, double rtol, int32_t maxit,
                 eqs_step_stats *st);

/* CG iterations of every stage of the last eqs_rkc_step (Sec. II: one
 * M-solve per stage), in stage order, for per-stage statistics (median,
 * spread) that eqs_step_stats' sum, minimum and maximum do not give. iters
 * (host) receives min(cap, n) entries and *n (may be NULL) the number of
 * stages whose solve ran in that step: s after a completed step, fewer after
 * a step that stopped on an error, 0 before the first step after a set-up
 * call (a call that its argument checks reject changes nothing). In a context
 * with several instances a stage's count is the largest over its instances.
 * EQS_ERR_INVALID_ARG for a NULL ctx, cap < 0, or iters NULL with cap > 0. */
int eqs_stage_iters(const eqs_ctx *ctx, int32_t *iters, int32_t cap, int32_t *n);

/* ---- error-controlled stepping -----------------------------------------
 * RKC with the step size and stage count chosen per step, as the paper runs
 * it (Sec. V: local time-integration error below a tolerance; the controller
 * is its ref. [9]'s). After a step of size tau from (t, y_n) to y_{n+1} the
 * local error is estimated as
 *   est = (12 (y_n - y_{n+1}) + 6 tau (F(t, y_n) + F(t + tau, y_{n+1}))) / 15
 * and measured as err = sqrt(mean_i (est_i / (atol + rtol max(|y_n,i|,
 * |y_{n+1},i|)))^2) over the free nodes; the step is accepted if err <= 1
 * (F(t + tau, y_{n+1}) is then the next step's first stage). The next size is
 * 0.8 tau err^(-1/3) after a rejection, tau max(0.1, min(10, 0.8 err^(-1/3)))
 * after the first accepted step and tau max(0.1, min(10, 0.8 (tau/tau_prev)
 * err_prev^(1/3) err^(-2/3))) after later ones, capped by tau_max and the end
 * of the interval. Each step takes the smallest s >= 2 whose stability
 * boundary covers it, beta(s) >= tau rho with rho = max over elements of
 * sigma_e / eps_e (sigma = kappa0 (1 + (alpha + 1)(|E|/e_s)^alpha), the
 * differential conductivity) at the step's start, an upper bound of the
 * spectral radius of M^-1 times the Jacobian of K(x)x; beyond s_max the step
 * is shortened to beta(s_max) / rho. */
typedef struct eqs_adapt_params {
    double atol;          /* absolute error weight (volts), > 0 */
    double rtol;          /* relative error weight, >= 0 */
    double tau0;          /* size of the first attempted step, > 0 */
    double tau_min;       /* smallest step allowed, >= 0 (a smaller one fails with EQS_ERR_STATE) */
    double tau_max;       /* largest step (0: t_end - t0) */
    int32_t s_max;        /* 2..256 [0: 256] */
    int32_t max_attempts; /* attempted steps before EQS_ERR_STATE [0: 100000] */
} eqs_adapt_params;

typedef struct eqs_adapt_record {
    double t;     /* start of the attempted step */
    double tau;   /* its size */
    double err;   /* its error norm */
    int32_t s;    /* its stages */
    int32_t accepted;
} eqs_adapt_record;

typedef struct eqs_adapt_stats {
    int32_t accepted;
    int32_t rejected;
    int32_t max_s;
    int32_t not_converged; /* stage solves that hit maxit */
    int64_t stages;        /* M-solves (one per stage, plus one per step for its end slope) */
    int64_t cg_iters;
    double last_tau;       /* the controller's next step size at t_end */
} eqs_adapt_stats;

/* Integrate from t0 to t_end with error-controlled RKC steps. x_dev (n_nodes
 * doubles) holds x(t0) on entry (Dirichlet entries ignored) and x(t_end) on
 * exit. Every M-solve runs CG to rtol from the previous solve's solution.
 * rec (host, may be NULL) receives the first cap attempted steps and *n_rec
 * (may be NULL) their total number; st may be NULL. Needs the plain or zero
 * start vector (EQS_ERR_STATE otherwise) and a single instance. Returns
 * EQS_ERR_NOT_CONVERGED if any solve hit maxit (the run still ends at
 * t_end). */
int eqs_rkc_adaptive(eqs_ctx *ctx, double t0, double t_end, double *x_dev, double rtol, int32_t maxit,
                     const eqs_adapt_params *p, eqs_adapt_record *rec, int32_t cap, int32_t *n_rec,
                     eqs_adapt_stats *st);

/* ---- batches of independent instances ---------------------------------
 * A context can hold several independent EQS problems at once (the batched
 * form): their meshes are concatenated (node ids of instance i in
 * [node_off[i], node_off[i+1]), its tets in [tet_off[i], tet_off[i+1])), and
 * materials and Dirichlet data are given for the concatenation as usual. The
 * element pass, the sparse products and the AMG hierarchy then act on all
 * instances at once (block-diagonal operators; aggregation never joins rows of
 * different instances), while every instance keeps its own CG scalars and its
 * own convergence test to rtol, so finished instances stop updating while the
 * others iterate. All instances share t, dt and s of eqs_rkc_step. Each
 * instance needs at least one Dirichlet node and, when n_inst > 1, at least
 * 256 free nodes. Call after eqs_set_mesh; invalidates the preconditioner. */
int eqs_set_instances(eqs_ctx *ctx, int32_t n_inst, const int64_t *node_off, const int64_t *tet_off);

/* Per-instance results of the last eqs_rkc_step or eqs_solve_M: CG iterations
 * (summed over the stages) and the largest final relative residual. Arrays of
 * n_inst entries (either may be NULL). */
int eqs_instance_stats(const eqs_ctx *ctx, int32_t n_inst, int64_t *iters, double *relres);

/* Convenience form: pack n contexts that hold mesh, materials and Dirichlet
 * data (same device; their own preconditioners are not needed) into one
 * batched context on `device`/`hip_stream`, built with p (NULL: defaults). */
typedef struct eqs_batch eqs_batch;
int eqs_batch_create(eqs_batch **out, int32_t n, eqs_ctx *const *ctxs, int device, void *hip_stream,
                     const eqs_amg_params *p);
int eqs_batch_destroy(eqs_batch *b);
/* eqs_set_graph_iters for the batch's packed context. */
int eqs_batch_set_graph_iters(eqs_batch *b, int32_t iters);
/* nsteps RKC(s) steps of every instance from t0 with step dt; x_dev[i] holds
 * instance i's n_nodes potentials (in/out, as eqs_rkc_step). st (may be NULL)
 * receives the batch's aggregated stats of the last step; per-instance
 * iterations through eqs_batch_instance_stats. */
int eqs_batch_rkc_steps(eqs_batch *b, int32_t nsteps, double t0, double dt, int32_t s, double *const *x_dev,
                        double rtol, int32_t maxit, eqs_step_stats *st);
int eqs_batch_instance_stats(const eqs_batch *b, int64_t *iters, double *relres);

/* ---- start vectors (Sec. IV) ------------------------------------------
 * The stage solves of one run form a multiple right-hand-side problem with the
 * constant M, so earlier solutions predict the next one (Sec. IV). Kinds:
 *   EQS_GUESS_PREVIOUS  the previous stage's solution (default)
 *   EQS_GUESS_ZERO      zero
 *   EQS_GUESS_GALERKIN  eq. (5) on the POD basis V of the last `window` stage
 *                       solutions: V (V^T M V)^{-1} V^T r (the reduced matrix
 *                       comes for free because M s_k = r_k for every stored
 *                       solution s_k)
 *   EQS_GUESS_MOR       eq. (5) on the POD basis of the first `window` stage
 *                       solutions, which is then kept for the rest of the run
 *                       (the reduced system is formed once; until the window
 *                       is full it behaves as GALERKIN)
 *   EQS_GUESS_MLP       F_{j-1} + V c, where the start-vector network
 *                       (eqs_mlp below) predicts the change c of the stage
 *                       solution on the same basis from the directions of
 *                       V^T F_{j-1} and of V^T (r_j - r_{j-1}); it is trained
 *                       online on the GPU from the run's own pairs, with
 *                       target V^T (F_j - F_{j-1}) once F_j is known.
 * For MLP a guard keeps the network's correction only if it lowers the M-norm
 * of the error of the start vector, which the reduced system gives without a
 * product with M (the Galerkin vector minimises that norm over a span holding
 * the previous solution, so it needs none); CG to rtol always follows, so the
 * start vector never changes the result beyond the solve tolerance. */
enum { EQS_GUESS_PREVIOUS = 0, EQS_GUESS_ZERO = 1, EQS_GUESS_GALERKIN = 2, EQS_GUESS_MLP = 3, EQS_GUESS_MOR = 4 };

#define EQS_MLP_NPARAM 7312 /* W1[64][32] b1[64] W2[64][64] b2[64] W3[16][64] b3[16], float */

typedef struct eqs_guess_params {
    int32_t kind;      /* EQS_GUESS_* */
    int32_t window;    /* window of stage solutions (and POD basis), 2..16 [16] */
    int32_t capacity;  /* replay-buffer pairs kept for training, <= 100000 [2000] */
    int32_t warmup;    /* pairs collected before the network's vector is used (0 = from the first pair) */
    int32_t batch;     /* training pairs drawn per stage, 1..256, in minibatches of up to 64 with one
                          Adam step each [256] */
    int32_t bf16;      /* 1: BF16 matmul operands, FP32 accumulation; 0: FP32 [1] */
    int32_t guard;     /* 1: keep the network's correction only where it lowers the error's M-norm [1] */
    int32_t add_threshold; /* GALERKIN, MOR: a stage solution joins the window only if its solve took
                              more than this many CG iterations (the first always joins) [0: every one] */
    double lr;         /* Adam learning rate [1e-3] */
    uint64_t seed;     /* minibatch sampling: SplitMix64 stream from this seed */
    const float *init; /* EQS_MLP_NPARAM initial parameters (host, copied); required for MLP */
} eqs_guess_params;

/* Select the start vector of every stage solve of eqs_rkc_step. Resets the
 * snapshot window, the replay buffer and (for MLP) the network. */
int eqs_set_guess(eqs_ctx *ctx, const eqs_guess_params *p);

/* The Galerkin start vector of eq. (5) (Sec. IV) on a window the caller
 * gives: x0 = V (V^T M V)^{-1} V^T r, V the POD basis of the k columns of S
 * (directions with singular values below 1e-7 of the largest dropped) and
 * V^T M V formed from R = M S (no product with M is taken here). The same
 * basis, reduced matrix and coefficient solve as a stage's
 * EQS_GUESS_GALERKIN start vector in eqs_rkc_step.
 * S_dev, R_dev: device, k x n_free doubles (column a at offset a * n_free,
 * oldest first), 1 <= k <= 16; r_dev, x0_dev: device, n_free doubles; x0
 * may not overlap S, R or r. Device pointers are borrowed for the call.
 * *m_out (host, may be NULL) receives the number of directions kept; with
 * none kept or a singular reduced matrix x0 = 0 and *m_out = 0. Runs on
 * the context's stream with its start-vector scratch and returns when x0
 * is written. Errors: EQS_ERR_INVALID_ARG (NULL, k, overlap),
 * EQS_ERR_STATE (before eqs_build_preconditioner). */
int eqs_galerkin_start(eqs_ctx *ctx, int32_t k, const double *S_dev, const double *R_dev, const double *r_dev,
                       double *x0_dev, int32_t *m_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as eqs_galerkin_start, with the same arguments and errors, but its
 * dot-product scratch is a static device array of the library (287,232 bytes
 * per GPU, held until the process ends) instead of context memory allocated
 * on first use; the call allocates nothing. k is limited to 16 (the scratch
 * holds the dots of 16 columns); a larger k gives EQS_ERR_INVALID_ARG. All
 * calls on one GPU share that array: calls that overlap in time on the same
 * GPU (other threads, other contexts' streams) race and must be serialised
 * by the caller. */
int eqs_galerkin_start_noalloc(eqs_ctx *ctx, int32_t k, const double *S_dev, const double *R_dev,
                               const double *r_dev, double *x0_dev, int32_t *m_out);

/* ---- the start-vector network on its own ------------------------------
 * Multilayer perceptron 32 -> 64 -> 64 -> 16, SiLU hidden activations,
 * linear output, mean-squared-error loss, Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8). One workgroup runs a minibatch (batch <= 64 for training).
 * Device arrays are row-major float: x[batch][32], y/t[batch][16]. */
typedef struct eqs_mlp eqs_mlp;

int eqs_mlp_create(eqs_mlp **out, int device, void *hip_stream, const float *params, int32_t bf16, double lr);
int eqs_mlp_destroy(eqs_mlp *net);
int eqs_mlp_forward(eqs_mlp *net, const float *x_dev, float *y_dev, int32_t batch);
/* One training step on the batch: loss, gradients, Adam update. *loss (host,
 * may be NULL) receives the batch loss before the update. */
int eqs_mlp_train_step(eqs_mlp *net, const float *x_dev, const float *t_dev, int32_t batch, float *loss);
/* Copy the FP32 master parameters and/or the last gradients to the host
 * (either pointer may be NULL; EQS_MLP_NPARAM floats each). */
int eqs_mlp_get(eqs_mlp *net, float *params_host, float *grad_host);

/* ---- per-kernel timing ------------------------------------------------
 * When enabled, the library records a pair of HIP events on the context's
 * stream around every launch of the selected kernel classes; durations are
 * summed at read time. Classes: */
enum {
    EQS_KCLASS_ELEMENT = 0,     /* fused element pass: K(x)x / stage right-hand side */
    EQS_KCLASS_SPMV_M = 1,      /* CG product q = M z + beta q (FP64 SpMV on M) */
    EQS_KCLASS_PRESMOOTH0 = 2,  /* finest-level Jacobi pre-smoothing + residual */
    EQS_KCLASS_POSTSMOOTH0 = 3, /* finest-level Jacobi post-smoothing (+ r.z) */
    EQS_KCLASS_VCYCLE = 4,      /* one whole V-cycle */
    EQS_KCLASS_CG_UPDATE = 5,   /* x += alpha p, r -= alpha q (+ |r|^2) */
    EQS_KCLASS_RKC_COMBINE = 6, /* RKC stage combination */
    EQS_KCLASS_RESTRICT0 = 7,   /* finest restriction b_1 = R_0 res (one product) */
    EQS_KCLASS_PROLONG0 = 8,    /* finest prolongation x_0 += P_0 x_1 (one product) */
    EQS_KCLASS_VCOARSE = 9,     /* all V-cycle work below the finest level (several kernels) */
    EQS_KCLASS_FINALISE = 10,   /* the one-block CG finalisers (three launches per iteration) */
    EQS_KCLASS_POSTSMOOTH1 = 11, /* level-1 Jacobi post-smoothing (when level 1 is not folded) */
    EQS_KCLASS_COUNT = 12
};

/* Enable timing of the classes whose bits are set in class_mask (bit k =
 * class k); 0 disables. Resets all counters. */
int eqs_profile_enable(eqs_ctx *ctx, uint32_t class_mask);

/* Launch count and summed duration (milliseconds) of one class since the last
 * eqs_profile_enable. Synchronises the context's stream. */
int eqs_profile_read(eqs_ctx *ctx, int32_t kclass, int64_t *launches, double *total_ms);

/* Text description of the built context (hierarchy sizes, the layout the
 * autotuner chose for every AMG operator): NUL-terminated, truncated to cap
 * bytes; *needed (may be NULL) receives the full length + 1. */
int eqs_describe(const eqs_ctx *ctx, char *buf, int64_t cap, int64_t *needed);

/* Message of the last failure on the calling thread ("" if none). */
const char *eqs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EQS_H */
