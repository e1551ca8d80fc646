/*
 * mfcg.h -- C-ABI of the MI355X (gfx950) fused matrix-free conjugate
 * gradient library.
 *
 * The library solves A u = b for the Q_k continuous finite-element
 * discretisation of the scalar Poisson problem -div(a grad u) = f on a
 * structured hexahedral mesh of [0,1]^3 deformed by an analytic map
 * (Kronbichler, Sashko, Munch, arXiv 2205.08909, Sec. 2, Eq. 1-5, in its
 * scalar form).  The operator is never assembled: every product with A is
 * the sum of cell integrals of Eq. 4/5 evaluated by sum factorisation.
 * The solver is the merged Jacobi-preconditioned CG of Algorithm 5 (Sec. 4.2)
 * whose vector updates ("pre") and seven inner products ("post") are
 * interleaved with the cell loop of the operator (Sec. 5), so that each
 * vector entry crosses HBM about once per iteration.
 *
 * Conventions shared by all entry points
 *  - Every function returns an int: MFCG_OK (0) or a negative MFCG_E* code.
 *    No C++ exception crosses this boundary.  mfcg_last_error() returns a
 *    human-readable description of the last failure on a handle.
 *  - Vectors are device pointers (caller owned, 8-byte aligned, on the
 *    handle's device) in lexicographic node order:
 *        i = gx + (nx*k + 1) * (gy + (ny*k + 1) * gz),
 *    gx in [0, nx*k], ...  The node count is (nx k+1)(ny k+1)(nz k+1) and
 *    includes the Dirichlet nodes (Sec. 5.3 keeps constrained unknowns in
 *    the linear system).
 *  - Cell-wise input is host memory, cell index c = cx + nx*(cy + ny*cz).
 *  - hip_stream is a hipStream_t passed as void* (NULL: the null stream).
 *    Calls are stream ordered; calls that return results on the host
 *    synchronise the stream before returning.
 *  - A handle owns all its device buffers; it is not thread safe: use one
 *    handle per host thread/stream.
 *  - Argument errors (MFCG_EINVAL) are detected before any HIP call.
 */
#ifndef MFCG_H
#define MFCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MFCG_OK = 0,
    MFCG_EINVAL = -1,      /* invalid argument (detected on the host, before any HIP call) */
    MFCG_ENOMEM = -2,      /* device allocation failed */
    MFCG_EHIP = -3,        /* a HIP runtime call failed */
    MFCG_ENOTCONV = -4,    /* maxit reached: x holds the last iterate */
    MFCG_EBREAKDOWN = -5,  /* p^T A p <= 0 or a non-finite scalar: operator not SPD or NaN input */
    MFCG_ESTAGNATION = -6  /* iterative refinement stopped reducing the residual */
};

enum {
    MFCG_MAP_AFFINE = 0,        /* x = X (Cartesian unit cube) */
    MFCG_MAP_SINE_SHEAR = 1,    /* x_i = X_i + A sin(2 pi X_{i+1}) sin(2 pi X_{i+2}) (indices mod 3) */
    MFCG_MAP_SINE_PRODUCT = 2   /* x_i = X_i + A prod_j sin(2 pi X_j) (keeps the unit cube) */
};

enum {
    MFCG_BC_DIRICHLET0 = 0,     /* boundary nodes are identity rows/columns of A */
    MFCG_BC_NONE = 1            /* no constraint (pure Neumann operator; singular) */
};

enum {
    MFCG_RHS_SINE = 0,          /* f = 3 pi^2 prod_j sin(pi x_j) */
    MFCG_RHS_BUMPS = 1          /* f = sum_m A_m exp(-|x - c_m|^2 / (2 s_m^2)) */
};

enum {
    MFCG_SOLVER_FUSED = 0,      /* Algorithm 5, pre/post fused into the operator's cell loop (default) */
    MFCG_SOLVER_ALG5_SPLIT = 1, /* Algorithm 5 as three passes: pre kernel, operator, post kernel */
    MFCG_SOLVER_PCG_BASIC = 2,  /* Algorithm 1: separate vector kernels and three reductions */
    MFCG_SOLVER_PIPELINED = 3,  /* Algorithm 2: pipelined CG, no preconditioner */
    MFCG_SOLVER_SSTEP = 4       /* Algorithm 3: s-step CG (monomial basis), no preconditioner */
};

enum {
    MFCG_PRECOND_JACOBI = 0,    /* M = diag(A), the point-Jacobi preconditioner (default) */
    MFCG_PRECOND_NONE = 1       /* M = I */
};

typedef struct mfcg_ctx *mfcg_handle;
typedef struct mfcg_batch_ctx *mfcg_batch;

/* Mesh: cells per direction on [0,1]^3, the map applied to it, the
 * boundary treatment. */
typedef struct {
    int32_t cells[3];
    int32_t map_kind;        /* MFCG_MAP_* */
    double map_amplitude;    /* A of the map; ignored for MFCG_MAP_AFFINE */
    int32_t bc;              /* MFCG_BC_* */
} mfcg_mesh;

/* Quadrature of the operator, the diagonal and the load vector. */
enum {
    MFCG_QUAD_GAUSS = 0, /* (k+1)^3 Gauss-Legendre points (default; the stored tensor of Sec. 2.2) */
    MFCG_QUAD_GLL = 1    /* (k+1)^3 Gauss-Lobatto-Legendre points = the nodes: collocation, the
                          * BP5 variation of Sec. 6; the interpolation passes drop out.  FP64 only:
                          * not with fp32 / mfcg_solve_ir, not in a batch */
};

/* Operator (Sec. 6's benchmark variations). */
enum {
    MFCG_OP_LAPLACE = 0, /* a_e grad u . grad v, Eq. 5 (default) */
    MFCG_OP_MASS = 1     /* a_e u v: the mass matrix of BP1 (scalar) and, through
                          * mfcg_solve_vector, BP2 (vector); Gauss points, FP64 only: not with
                          * fp32 / mfcg_solve_ir, not in a batch */
};

/* Geometry representation of the operator (Sec. 2.2). */
enum {
    MFCG_GEOM_STORED = 0,   /* G_q = a_e w_q det J_q J_q^{-1} J_q^{-T} stored per quadrature point and read
                             * by every mat-vec ("final tensor load"; default) */
    MFCG_GEOM_QUADRATIC = 1 /* quadratic geometry: per cell the map's values at the 27 points
                             * (c + (a, b, d) / 2) / n and a_e are stored (82 doubles); the mat-vec
                             * evaluates J_q of their quadratic interpolant at each Gauss point and forms
                             * G_q on the fly.  The operator is that of the interpolated map (diagonal and
                             * load vector too).  Laplacian or mass operator on k+1 or k+2 Gauss points,
                             * FP64: not with GLL, fp32 / mfcg_solve_ir or a batch; the vector solve
                             * evaluates the geometry once per component */
};

/* Options.  Zero-initialised fields select the defaults. */
typedef struct {
    int32_t n_q_1d;          /* Gauss points per direction: 0 or k+1 (default), or k+2 (the
                              * n_q = (k+2)^3 rule of the BP1-BP4 benchmarks of Sec. 6; k <= 7,
                              * Gauss only, FP64 only: not with fp32 / mfcg_solve_ir, not in a
                              * batch; the stored tensor grows to (k+2)^3 points per cell) */
    int32_t tile[3];         /* cells per tile in x, y, z; 0: per-degree default.  x and y at most
                              * the fused kernel's compiled extent, (x, y) = (8, 8), (8, 8),
                              * (8, 4), (4, 4), (4, 3), (2, 2), (2, 2), (2, 1) for k = 1..8, which
                              * is also the default; default z 16 */
    int32_t check_every;     /* iterations between host polls of the convergence flag; 0: 16 */
    int32_t fp32;            /* 1: build the FP32 operator copy of mfcg_solve_ir at set-up (else on first use) */
    int32_t quad_rule;       /* MFCG_QUAD_* */
    int32_t op;              /* MFCG_OP_* */
    int32_t geometry;        /* MFCG_GEOM_* */
    int32_t deterministic;   /* accepted for interface compatibility; 0 and 1 behave the same: every
                              * reduction and every sum of partial contributions runs in a fixed
                              * order (no floating-point atomics), so results are always bitwise
                              * reproducible from run to run on the same device */
    const char *tune_cache;  /* mfcg_setup_batch: path of the autotuner cache (JSON, one record per
                              * GPU, degree, tuning cube size, map and precision; created or updated
                              * in place; a record whose tile exceeds this build's compiled x/y
                              * extent is tuned again and replaced); NULL: tune on every call.
                              * Ignored by mfcg_setup */
} mfcg_options;

/* Builds the operator (Sec. 2, Eq. 3-5): tiles and DoF enumeration of the
 * fused loop (Sec. 5.3), the stored per-quadrature-point tensor
 * G_q = a_e w_q det(J_q) J_q^{-1} J_q^{-T} (the "final tensor load"
 * variant of Sec. 2.2), and the Jacobi diagonal (Sec. 3).
 *   degree      polynomial degree k, 1..8
 *   cell_coeff  host, nx*ny*nz positive finite values a_e; NULL: a = 1
 *   opt         NULL: defaults
 * Errors: EINVAL (null mesh/out, cells < 1, degree out of range, bad map or
 * bc, non-positive coefficient, unsupported n_q_1d, tile < 0 or beyond the
 * compiled x/y extent), ENOMEM, EHIP.
 * On error *out is NULL. */
int mfcg_setup(const mfcg_mesh *mesh, int32_t degree, const double *cell_coeff,
               const mfcg_options *opt, void *hip_stream, mfcg_handle *out);

/* Replaces the cell coefficient a_e (host, nx*ny*nz positive finite values
 * as in mfcg_setup; NULL: a = 1) and rebuilds G_q and the diagonal (and the
 * FP32 copy if one exists) without rebuilding the enumeration.  Must not
 * be called between mfcg_cg_begin and mfcg_cg_end.  Synchronises
 * hip_stream.  Errors: EINVAL, ENOMEM, EHIP. */
int mfcg_set_coefficient(mfcg_handle h, const double *cell_coeff, void *hip_stream);

/* Initial guess from a predicted solution shape u (device, lexicographic):
 * the Galerkin-optimal multiple x0 = s u', s = u'^T b / u'^T A u', where u'
 * is u with its Dirichlet entries set to 0.  This minimises the A-norm of
 * the error over multiples of u', so ||x* - x0||_A <= ||x*||_A: never
 * worse than x0 = 0 in the norm CG minimises (Sec. 3).  x0 = 0 instead if
 * u'^T A u' is not positive or s is 0 or not finite, or if
 * ||b - A x0|| >= max_rel_res ||b|| (pass +inf to accept any residual).
 *   x0       device out, lexicographic, may not alias b or u
 *   scale    host out or NULL: s (0 when x0 = 0)
 *   rel_res  host out or NULL: ||b - A x0|| / ||b|| (1 when x0 = 0)
 *   used     host out or NULL: 1 if x0 = s u', 0 if x0 = 0
 * Uses the handle's work vectors: must not be called between
 * mfcg_cg_begin and mfcg_cg_end.  Synchronises hip_stream.
 * Errors: EINVAL (null pointers, max_rel_res NaN), EHIP. */
int mfcg_warmstart(mfcg_handle h, const double *b, const double *u, double max_rel_res, double *x0, double *scale,
                   double *rel_res, int32_t *used, void *hip_stream);

/* The same guarantee over a span (Sec. 3, CG minimises the A-norm of the
 * error): x0 = sum_i c_i u_i', the u_i' being the m vectors u_i with their
 * Dirichlet entries set to 0, with the coefficients that minimise
 * ||x - x0||_A over their span (the Galerkin system G c = g, G_ij =
 * u_i'^T A u_j', g_i = u_i'^T b, solved by Cholesky in the given order; a
 * vector whose pivot is not above 1e-12 u_i'^T A u_i' -- zero, or in the
 * span of the earlier ones -- gets c_i = 0).  So x0 is never worse in the
 * A-norm than the best Galerkin-scaled single u_i, nor than x0 = 0.  With
 * m = 1 it is mfcg_warmstart.
 *   m        1 <= m <= MFCG_SPAN_MAX
 *   u        host array of m device vectors (lexicographic, length n)
 *   coef     host out or NULL: m coefficients (all 0 when x0 = 0)
 *   other arguments and the fall-back to x0 = 0 as for mfcg_warmstart.
 * Allocates 2 m n doubles of work vectors the first time m grows (kept by
 * the handle).  Must not be called between mfcg_cg_begin and mfcg_cg_end.
 * Synchronises hip_stream.  Errors: EINVAL (null pointers, m out of range,
 * max_rel_res NaN), ENOMEM, EHIP. */
#define MFCG_SPAN_MAX 8
int mfcg_warmstart_span(mfcg_handle h, const double *b, int32_t m, const double *const *u, double max_rel_res,
                        double *x0, double *coef, double *rel_res, int32_t *used, void *hip_stream);

/* Interpolation between two handles on the same cells (Sec. 2: the
 * continuous Q_k space with its nodes at the Gauss-Lobatto points of every
 * cell): dst = the Q_{k_from} finite-element function with nodal values
 * src, evaluated at the nodes of the Q_{k_to} space of handle `to`.  For
 * k_from <= k_to the spaces are nested and this is their exact embedding
 * (e.g. a Q1 solution as a Q3 vector, the coarse level of a two-level
 * initial guess).  The evaluation is per cell in reference coordinates, so
 * it does not depend on the mesh map; nodes on cell faces take the value
 * both sides share.
 *   src  device, lexicographic nodal values of `from` (its n)
 *   dst  device out, lexicographic, the n of `to`; may not alias src
 * Synchronises hip_stream.  Errors: EINVAL (null pointers, different cell
 * counts, src == dst), EHIP. */
int mfcg_interpolate(mfcg_handle from, const double *src, mfcg_handle to, double *dst, void *hip_stream);

/* Number of nodes (vector length), Dirichlet nodes included. */
int mfcg_n_dofs(mfcg_handle h, int64_t *n);

/* dst = A src (Eq. 4): the matrix-free operator, identity rows on Dirichlet
 * nodes.  dst and src are distinct device vectors of length n_dofs. */
int mfcg_vmult(mfcg_handle h, double *dst, const double *src, void *hip_stream);

/* diag = diag(A) (the point-Jacobi preconditioner, Sec. 3); 1 on Dirichlet
 * nodes.  Device vector of length n_dofs. */
int mfcg_diagonal(mfcg_handle h, double *diag, void *hip_stream);

/* dst = A32 src with the single-precision operator of mfcg_solve_ir (the
 * inner solver of the mixed-precision extension: G_q stored in FP32, the
 * sum factorisation and the sums in FP32): src rounded to FP32, the result
 * widened to FP64; lexicographic device vectors as mfcg_vmult.  Builds the
 * FP32 copy on first use and uses its work vectors (no solve may be in
 * progress on the handle).  Gauss-point Laplacian with the stored tensor
 * only.  Errors: EINVAL (null or aliasing vectors, other operators), ENOMEM,
 * EHIP. */
int mfcg_vmult_fp32(mfcg_handle h, double *dst, const double *src, void *hip_stream);

/* Load vector b_i = sum_e sum_q f(x_q) phi_i(x_q) w_q det J_q on free nodes,
 * 0 on Dirichlet nodes, Gauss quadrature with k+1 points per direction.
 *   kind    MFCG_RHS_*
 *   params  host; MFCG_RHS_BUMPS: [nb, (A, cx, cy, cz, s) x nb], nb <= 64;
 *           ignored for MFCG_RHS_SINE. */
int mfcg_assemble_rhs(mfcg_handle h, int32_t kind, const double *params, double *b, void *hip_stream);

/* Jacobi-preconditioned CG, Algorithm 5 with the vector updates and inner
 * products fused into the operator's cell loop (Sec. 4.2, Sec. 5).
 *   b, x           device vectors; x holds x_0 on entry and the solution on
 *                  return (also on ENOTCONV: the last iterate)
 *   tol            stop when the residual norm ||r_j||_2 < tol * ||b||_2
 *                  (Sec. 3.1 terminates on the unpreconditioned residual);
 *                  tol = 0 runs exactly maxit iterations
 *   maxit          >= 1
 *   iters          host out: iterations performed (matrix-vector products)
 *   res_hist       host, maxit+1 doubles or NULL: res_hist[0] = ||r_0||,
 *                  res_hist[j] = the residual norm after iteration j as
 *                  predicted by Eq. 8 (the algorithm's own stopping value)
 *   true_rel_res   host or NULL: ||b - A x||_2 / ||b||_2 recomputed after
 *                  the solve (costs one operator application)
 * ||b|| = 0 returns x = 0, *iters = 0, MFCG_OK.
 * Errors: EINVAL (null pointers, tol < 0 or not finite, maxit < 1),
 * ENOTCONV, EBREAKDOWN, EHIP.  Synchronises hip_stream. */
int mfcg_solve(mfcg_handle h, const double *b, double *x, double tol, int32_t maxit,
               int32_t *iters, double *res_hist, double *true_rel_res, void *hip_stream);

/* The vector-valued Poisson problem of the paper's benchmark (Sec. 2, Eq. 1;
 * BP4): three uncoupled components u = (u_x, u_y, u_z), each with the
 * handle's scalar operator, so the system is I_3 (x) A with the one scalar
 * diagonal applied to all components (Sec. 3), I_3 (x) diag(A), and it is
 * solved by one CG (Algorithm 5; every inner product runs over all 3n
 * entries).  Each iteration is one launch of the fused tile kernel over
 * (tile, component) pairs -- a tile's three components run side by side,
 * so the geometry tensor they share is read from HBM about once -- the
 * shared-node kernel per component and one finish over all components'
 * inner-product records.  The operator is the handle's: the Laplacian on
 * (k+1)^3 or (k+2)^3 Gauss points (BP4), with the stored tensor or the
 * quadratic geometry (evaluated once per component), GLL collocation, or
 * the mass operator (BP2).
 *   b, x   device vectors of 3n doubles, component-blocked: entries
 *          [c*n, (c+1)*n) hold component c in lexicographic node order;
 *          x holds x_0 on entry and the solution on return
 *   other arguments, the stopping rule and res_hist as for mfcg_solve.
 * Allocates 4 work vectors of 3n doubles at the first call.  Ends a
 * stepping-interface solve in progress (its state is reused): call
 * mfcg_cg_begin again before mfcg_cg_iterate.
 * Errors: EINVAL (null pointers, tol < 0 or not finite, maxit < 1),
 * ENOTCONV, EBREAKDOWN, ENOMEM, EHIP.  Synchronises hip_stream. */
int mfcg_solve_vector(mfcg_handle h, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                      double *res_hist, double *true_rel_res, void *hip_stream);

/* Many right-hand sides on one operator (an extension of Algorithm 5, Sec.
 * 4.2): m independent solves A x_c = b_c, c = 0..m-1, each with its own CG
 * scalars and its own stopping test ||r_c||_2 < tol ||b_c||_2.  One fused
 * launch per iteration covers every (tile, right-hand side) pair, the
 * right-hand side index fastest, so a tile's geometry tensor G_q is read
 * from HBM about once per iteration for all m; a right-hand side that has
 * stopped drops out while the others go on.
 *   m         1 <= m <= MFCG_MULTI_MAX
 *   b, x      host arrays of m device pointers, each a vector of n doubles
 *             in lexicographic node order; x[c] holds x_0 on entry and the
 *             solution on return.  A zero b[c] gives x[c] = 0, 0 iterations.
 *   iters     host, m: iterations taken by each
 *   status    host, m: MFCG_OK, MFCG_ENOTCONV or MFCG_EBREAKDOWN
 *   true_rel_res  host, m doubles or NULL: ||b_c - A x_c|| / ||b_c||
 * Each right-hand side follows exactly the iteration of mfcg_solve with the
 * Jacobi preconditioner on this handle's operator variant.  Allocates 4 m n
 * doubles of work vectors at the first call with this m or a larger one,
 * and m (maxit + 1) doubles of residual history when maxit grows (both
 * kept by the handle; ENOMEM when the device cannot hold them, after which
 * the handle stays usable).  Ends a stepping-interface solve in progress.
 * Returns MFCG_OK when every right-hand side converged, else the first
 * non-OK status (ENOTCONV or EBREAKDOWN; the per-right-hand-side results
 * are filled in either case); EINVAL for bad arguments; ENOMEM, EHIP.
 * Synchronises hip_stream. */
#define MFCG_MULTI_MAX 64
int mfcg_solve_multi(mfcg_handle h, int32_t m, const double *const *b, double *const *x, double tol, int32_t maxit,
                     int32_t *iters, int32_t *status, double *true_rel_res, void *hip_stream);

/* Mixed precision: FP64 iterative refinement around the fused solver run
 * in FP32 (operator with an FP32 copy of G_q and D^{-1}, vector updates and
 * inner products in FP32).  Outer loop in FP64 on the GPU:
 *     r = b - A x (FP64 operator); stop when ||r||_2 < tol ||b||_2;
 *     solve A d = r in FP32 until its recursive residual is below
 *     max(inner_tol, tol ||b|| / (2 ||r||)) ||r|| (checked every 16
 *     iterations; the second bound stops the last inner solve at what the
 *     outer target needs) or max_inner iterations; x += d (FP64).
 *   keep_direction  0: every inner solve is a fresh CG (classical
 *                   refinement).  1: after the first, each inner solve
 *                   continues the previous search direction with the
 *                   replaced FP64 residual, p = D^{-1} r + beta p_prev (CG
 *                   with residual replacement, "reliable updates"): the
 *                   Krylov information survives the corrections.  A
 *                   correction that reduced the residual less than 10x
 *                   restarts the direction.
 *   x          device, x_0 on entry, solution on return
 *   outer_its  host out: corrections applied; inner_its: FP32 iterations summed
 *   res_hist   host or NULL, max_outer+1 doubles: ||b - A x_j|| / ||b||
 *   true_rel_res host or NULL: the final ||b - A x|| / ||b|| (FP64)
 * Errors: EINVAL (tol <= 0, inner_tol not in (0,1), max_* < 1), ENOTCONV
 * (max_outer corrections without reaching tol), ESTAGNATION (the outer
 * residual decreased by less than 10x in two consecutive corrections),
 * EBREAKDOWN, EHIP.  The first call builds the FP32 copy (half the geometry
 * bytes) unless mfcg_options.fp32 asked for it at set-up. */
int mfcg_solve_ir(mfcg_handle h, const double *b, double *x, double tol, double inner_tol, int32_t max_outer,
                  int32_t max_inner, int32_t keep_direction, int32_t *outer_its, int32_t *inner_its,
                  double *res_hist, double *true_rel_res, void *hip_stream);

/* Stepping interface used for throughput measurement: mfcg_cg_begin
 * initialises the solver state from (b, x0) exactly as mfcg_solve does;
 * mfcg_cg_iterate enqueues n fused iterations (no host synchronisation;
 * iterations after convergence are no-ops); mfcg_cg_end reconstructs the
 * final x (Algorithm 5's delayed x update) into x and returns the
 * iteration count and status.  Timing: when mfcg_set_timing(h, 1) is on,
 * every launch of the fused cell kernel and of the shared-node kernel is
 * bracketed by HIP events on hip_stream; mfcg_get_timing returns the summed
 * milliseconds and launch counts since the last reset. */
int mfcg_cg_begin(mfcg_handle h, const double *b, const double *x0, double tol, int32_t maxit,
                  void *hip_stream);
int mfcg_cg_iterate(mfcg_handle h, int32_t n, void *hip_stream);
int mfcg_cg_end(mfcg_handle h, double *x, int32_t *iters, double *res_hist, void *hip_stream);
int mfcg_set_timing(mfcg_handle h, int32_t enable);
int mfcg_get_timing(mfcg_handle h, double *fused_ms, int64_t *fused_launches, double *shared_ms,
                    int64_t *shared_launches);

/* Selects the iteration used by mfcg_solve and the stepping interface
 * (MFCG_SOLVER_*); it takes effect at the next mfcg_cg_begin / mfcg_solve.
 * The comparison solvers apply the same operator kernels in plain mat-vec
 * mode and move the vector updates and inner products into separate
 * streaming kernels:
 *  - Algorithm 5 split into its pre / operator / post regions (Sec. 4.2,
 *    the paper's GPU scheme of Sec. 6) and the textbook Jacobi-PCG of
 *    Algorithm 1 (Sec. 3): the iterates of the fused solver in exact
 *    arithmetic;
 *  - pipelined CG (Algorithm 2, Sec. 4.1): one mat-vec q = A w, then one
 *    loop-fused kernel for the six vector updates and the two inner
 *    products; stops on the recursively updated ||r||;
 *  - s-step CG (Algorithm 3, Sec. 4.1, monomial basis, s from
 *    mfcg_set_sstep): per phase of s iterations, s + 1 mat-vecs and four
 *    vector passes with block inner products and s x s solves; stops on the
 *    true residual ||b - A x|| checked at the end of each phase.  Iteration
 *    counts are multiples of s; a phase runs only if it ends within maxit,
 *    res_hist holds NaN inside a phase.  The monomial basis loses
 *    orthogonality as s and the condition number grow (the paper's caveat),
 *    so it may stall or break down (MFCG_EBREAKDOWN) where CG converges.
 *  The last two are unpreconditioned, as the paper compares them, and need
 *  3 (pipelined) or 2s+1 (s-step) extra vectors of n doubles, allocated at
 *  the first mfcg_cg_begin that uses them.  Timing events cover
 *  MFCG_SOLVER_FUSED only; the FP32 refinement, the warm start and the
 *  batch always use the fused solver.
 * Errors: EINVAL (null handle, unknown solver). */
int mfcg_set_solver(mfcg_handle h, int32_t solver);

/* Preconditioner of the solvers that take one (MFCG_PRECOND_*): with
 * MFCG_PRECOND_NONE the fused solver runs Algorithm 4 (the merged CG of
 * Sec. 4.2, the same kernels with the diagonal never read), the split
 * solver Algorithm 4 in three passes and the basic solver the textbook CG
 * (Algorithm 1 with z = r).  Pipelined and s-step CG never precondition;
 * the FP32 refinement, the warm start and the batch always use Jacobi.
 * Takes effect at the next begin.
 * Errors: EINVAL (null handle, unknown value). */
int mfcg_set_preconditioner(mfcg_handle h, int32_t precond);

/* Block size s of MFCG_SOLVER_SSTEP (Algorithm 3), 1..8; default 6, the
 * value of the paper's comparison.  Takes effect at the next begin.
 * Errors: EINVAL (null handle, s out of range). */
int mfcg_set_sstep(mfcg_handle h, int32_t s);

/* Layout facts of the handle (host out, any may be NULL): tile sizes in
 * cells, node counts of the classes of the enumeration (tile-interior,
 * shared between tiles, Dirichlet), tile count, bytes of the stored
 * geometry tensor. */
int mfcg_layout_info(mfcg_handle h, int32_t *tile, int64_t *n_interior, int64_t *n_shared,
                     int64_t *n_dirichlet, int64_t *n_tiles, int64_t *geometry_bytes);

/* Host-only: the lexicographic -> internal permutation the library would
 * use for this mesh, degree and tile (tile entries 0: defaults), written to
 * perm[n_dofs] (host), and the class counts.  No HIP call. */
int mfcg_layout_permutation(const mfcg_mesh *mesh, int32_t degree, const int32_t *tile, int64_t *perm,
                            int64_t *n_interior, int64_t *n_shared, int64_t *n_dirichlet);

/* Streaming reference kernels giving the device's measured bandwidth
 * ceiling (the denominator of the "measured" roofline and the calibration
 * kernel of the HBM byte counters).  kind 0: dst[0..n) = src[0..n) (one read
 * and one write per element); kind 1: dst[b] = partial sum of src over block
 * b of the grid (one read per element; dst holds nblocks doubles).  Bits 1-2
 * of kind: log2 of the independent 16-byte loads each thread keeps in flight
 * (1, 2 or 4; 3 is invalid); bit 3: non-temporal hint on loads and stores.
 * n even, 16-byte aligned device pointers; nblocks >= 1 workgroups of 256
 * threads. */
int mfcg_stream_bench(int32_t kind, int64_t n, const double *src, double *dst, int32_t nblocks, void *hip_stream);

/* Tile autotuner: times `iters` fused iterations (after 2 untimed ones)
 * of a Poisson problem on `mesh` for each candidate tile and returns the
 * fastest in tile_out[3] and its time per iteration in *ms_out (may be
 * NULL).  Candidates: the compiled maximum extent in x and y with 8, 16 or
 * 32 cell layers in z or the mesh's z extent split into 1..12 equal tile
 * layers (2..64 cells deep), and half the x/y extent with 16 layers; all
 * clipped to the mesh.  Builds and frees one handle per
 * candidate.  Errors: EINVAL, ENOMEM, EHIP. */
int mfcg_autotune_tile(const mfcg_mesh *mesh, int32_t degree, int32_t iters, int32_t *tile_out, double *ms_out,
                       void *hip_stream);

/* Batches of independent problems of different sizes and degrees solved
 * together.  In every CG iteration of the batch, the problems too small to
 * fill the device (fewer than 512 tiles) are packed: one launch of the
 * fused tile kernel per degree present over a work list of
 * (problem, tile) items, one shared-node launch over (problem, block)
 * items and one finish launch with a block per problem; each larger
 * problem runs its own three launches.  Each problem keeps its own scalars
 * and convergence test (its own Algorithm 5 iteration, identical to
 * mfcg_solve's, bitwise), and problems that have converged drop out of the
 * work lists at the next poll (every 16 iterations).
 *   meshes, degrees  nprob entries (as for mfcg_setup)
 *   coeffs           host array of nprob host pointers (entries or the
 *                    array itself NULL: a = 1)
 *   autotune         1: one tile per degree from mfcg_autotune_tile on a
 *                    cube of min(largest cells, 48) cells; 0: defaults
 * Errors: EINVAL (the failing problem is named in the message), ENOMEM,
 * EHIP.  On error *out is NULL. */
int mfcg_batch_setup(int32_t nprob, const mfcg_mesh *meshes, const int32_t *degrees, const double *const *coeffs,
                     int32_t autotune, void *hip_stream, mfcg_batch *out);

/* Problem i of the batch: its handle (owned by the batch; valid for
 * mfcg_vmult, mfcg_diagonal, mfcg_assemble_rhs, mfcg_n_dofs...) and the
 * tile it uses; either output may be NULL. */
int mfcg_batch_info(mfcg_batch hb, int32_t i, mfcg_handle *h, int32_t *tile);

/* Solves all problems to ||r_i|| < tol ||b_i|| (each as mfcg_solve would)
 * or maxit iterations.  b, x: host arrays of nprob device pointers (x: x0
 * in, solution out).  iters, status: host arrays of nprob (status: MFCG_OK,
 * MFCG_ENOTCONV or MFCG_EBREAKDOWN per problem).  Returns MFCG_OK if every
 * problem converged, else the first non-OK status; EINVAL/EHIP on errors.
 * Synchronises hip_stream. */
int mfcg_batch_solve(mfcg_batch hb, const double *const *b, double *const *x, double tol, int32_t maxit,
                     int32_t *iters, int32_t *status, void *hip_stream);
/* The batch calls under the names of the library's interface summary:
 * mfcg_setup_batch takes mfcg_options (NULL: defaults) instead of the
 * autotune flag: a tile with all three extents > 0 is used for every
 * problem (clipped to its mesh), otherwise one tile per degree is tuned,
 * read from and written to opt->tune_cache when that is set; the other
 * option fields must be 0 (a batch runs the FP64 Gauss-point Laplacian
 * with the stored tensor).  mfcg_solve_batch is mfcg_batch_solve. */
int mfcg_setup_batch(int32_t nprob, const mfcg_mesh *meshes, const int32_t *degrees, const double *const *coeffs,
                     const mfcg_options *opt, void *hip_stream, mfcg_batch *out);
int mfcg_solve_batch(mfcg_batch hb, const double *const *b, double *const *x, double tol, int32_t maxit,
                     int32_t *iters, int32_t *status, void *hip_stream);
int mfcg_batch_destroy(mfcg_batch hb);
const char *mfcg_batch_last_error(mfcg_batch hb);

int mfcg_destroy(mfcg_handle h);
const char *mfcg_error_string(int code);
const char *mfcg_last_error(mfcg_handle h);

#ifdef __cplusplus
}
#endif
#endif
