/* kernels.h -- launch wrappers of the gfx950 kernels (host callable). */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mfcg_internal.h"

namespace mfcg {

/* MODE_CG: one iteration of Algorithm 5 with the Jacobi preconditioner;
 * MODE_CG_NOPREC: the same with M = I (Algorithm 4, the merged CG), the
 * diagonal never read; MODE_VMULT: dst = A src. */
enum Mode : int { MODE_CG = 0, MODE_VMULT = 1, MODE_CG_NOPREC = 2 };
constexpr bool mode_is_cg(int m) { return m != MODE_VMULT; }
/* or-ed into the mode argument of launch_fused (FP64 only): quadrature on
 * the GLL nodes (collocation) instead of the Gauss points */
constexpr int MODE_GLL = 8;
/* or-ed likewise: the mass operator (Gauss points; FP64 only) */
constexpr int MODE_MASS = 16;
/* or-ed likewise: k + 2 Gauss points per direction instead of k + 1
 * (k <= 7, Laplacian or mass; FP64 only) */
constexpr int MODE_Q2 = 32;
/* or-ed likewise: quadratic geometry evaluated in the kernel (Laplacian or
 * mass operator, Gauss points, FP64): the geometry argument is the per-cell
 * node array below instead of the stored tensor */
constexpr int MODE_QGEOM = 64;
/* doubles per cell of the quadratic geometry array: the 27 interpolation
 * points' coordinates (x, y and z blocks of 27, point a + 3 b + 9 d at
 * reference position (a, b, d) / 2) and a_e */
constexpr int QGEOM_STRIDE = 82;

/* Arguments of the fused tile kernel and the shared-node kernel. */
template <typename T>
struct IterArgs {
    LayoutView L;
    const T *G;     /* geometry tensor, tile-blocked */
    const T *dinv;  /* inverse diagonal, internal order (1 on Dirichlet nodes) */
    T *r, *p, *v, *x;
    const T *src;   /* MODE_VMULT input */
    T *dst;         /* MODE_VMULT output */
    T *part;        /* shared-node partial sums */
    T *dots;        /* per-block partial inner products, 8 per block */
    CGState *st;
    double *hist;
    int32_t nshared_blocks;
};

/* One CG iteration of a batch of independent problems (device work lists):
 * per degree K, items[K][0..nitems[K]) = (problem, tile) pairs for the
 * fused tile kernel; shared_items = (problem, block) pairs for the
 * shared-node kernel; active = the problems whose finish runs. */
struct BatchLaunch {
    const IterArgs<double> *probs;
    const int2 *items[9];
    int nitems[9];
    const int2 *shared_items;
    int nshared_items;
    const int *active;
    int nactive;
};
hipError_t launch_batch_iteration(const BatchLaunch &b, hipStream_t s);
/* out[i] = *probs[i].st, i < np (one launch instead of np small copies) */
hipError_t launch_gather_states(const IterArgs<double> *probs, int np, CGState *out, hipStream_t s);

/* Maximum tile extent in x and y (cells) compiled for degree K. */
void tile_limits(int K, int *tx, int *ty);
int fused_block_size(int K);

template <typename T>
hipError_t launch_fused(int K, int mode, const IterArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_shared(int mode, const IterArgs<T> &a, hipStream_t s);
/* Vector problems (several components sharing the operator): the
 * shared-node kernel of one component without the finish, and the finish
 * over nparts records starting at a.dots (all components' records). */
hipError_t launch_shared_nofinish(const IterArgs<double> &a, hipStream_t s);
/* Independent right-hand sides c = 0..m-1 on one operator (vectors at
 * c*nstride, partial sums at c*pstride, records at c*dstride, state a.st + c,
 * history at c*hstride): the shared-node kernel over (block, c) and one
 * finish block per c; a right-hand side whose CG has stopped is skipped. */
hipError_t launch_shared_finish_multi(const IterArgs<double> &a, int m, int64_t nstride, int64_t pstride,
                                      int64_t dstride, int64_t hstride, hipStream_t s);
/* The fused tile kernel over all three components of a vector problem in
 * one launch (mode: MODE_CG, optionally with MODE_GLL, MODE_MASS or
 * MODE_QGEOM, and MODE_Q2 without MODE_GLL); the
 * vectors, shared partial sums and records of component c sit at c times
 * the given strides (elements). */
hipError_t launch_fused_vec(int K, int mode, const IterArgs<double> &a, int m, int64_t nstride, int64_t pstride,
                            int64_t dstride, int sstride, hipStream_t s);
hipError_t launch_finish_parts(const IterArgs<double> &a, int64_t nparts, hipStream_t s);

/* Setup kernels (FP64). */
struct GeomArgs {
    LayoutView L;
    Tables<double> tab;
    int32_t K, map_kind;
    double amp;
    int32_t bc;
    const double *coeff; /* per cell, device */
    int32_t op;          /* 0: Laplacian (6-component tensor), 1: mass (component 0: a_e w_q det J_q) */
    int32_t nq;          /* quadrature points per direction (k + 1 or k + 2); tab.S, tab.Sd are nq x (k+1), tab.D nq x nq */
    const double *X;     /* quadratic geometry per cell (QGEOM_STRIDE doubles, tile-blocked like G), device; NULL:
                          * the map itself */
};
hipError_t launch_geometry(const GeomArgs &g, double *G, hipStream_t s);
/* The quadratic geometry array X (QGEOM_STRIDE doubles per cell, tile-blocked:
 * a tile's cells after those of earlier tiles, layer by layer, x fastest):
 * the map at the 27 interpolation points of each cell and a_e. */
hipError_t launch_qgeom_nodes(const GeomArgs &g, double *X, hipStream_t s);
hipError_t launch_diagonal(const GeomArgs &g, const double *G, double *diag_lex, double *dinv_int, hipStream_t s);
hipError_t launch_rhs(const GeomArgs &g, int kind, const double *params, int nparams, double *b_lex, hipStream_t s);

/* Vector utilities. */
template <typename T>
hipError_t launch_lex_to_int(const LayoutView &L, const double *in_lex, T *out_int, hipStream_t s);
template <typename T>
hipError_t launch_int_to_lex(const LayoutView &L, const T *in_int, double *out_lex, hipStream_t s);
/* r = r - v (use_v), p = 0, v = 0 */
hipError_t launch_init_cg(int64_t n, double *r, double *p, double *v, int use_v, hipStream_t s);
/* dinv == NULL: unit diagonal (no preconditioner) */
template <typename T>
hipError_t launch_reconstruct(int64_t n, T *x, const T *p, const T *r, const T *dinv, const CGState *st,
                              hipStream_t s);
/* part[0..nb) = block sums of (a_i - c_i)^2 (c may be NULL); the caller adds them in order */
hipError_t launch_sumsq(int64_t n, const double *a, const double *c, double *part, int nb, hipStream_t s);
hipError_t launch_convert(int64_t n, const double *in, float *out, hipStream_t s);
/* part[0..nb) = block sums of a_i b_i (mode 0) or (a_i - sc b_i)^2 (mode 1) */
hipError_t launch_pair_sum(int64_t n, int mode, const double *a, const double *b, double sc, double *part, int nb,
                           hipStream_t s);
/* out = sc a */
hipError_t launch_scale(int64_t n, const double *a, double sc, double *out, hipStream_t s);
/* dst (Q_kt nodal values, lexicographic) = the Q_kf function src
 * (lexicographic) at the Q_kt nodes of the same cells; W[i (kf+1) + j] =
 * the j-th degree-kf Lagrange basis function on the GLL nodes at the i-th
 * degree-kt GLL node */
struct InterpArgs {
    int32_t ncells[3];
    int32_t kf, kt;
    double W[MAXN * MAXN];
    const double *src;
    double *dst;
};
hipError_t launch_interpolate(const InterpArgs &a, hipStream_t s);
/* out = sum_{i < m} c_i U_i, U_i = U + i n */
constexpr int LINCOMB_MAX = 8;
struct LinComb {
    double c[LINCOMB_MAX];
};
hipError_t launch_lincomb(int64_t n, int m, const double *U, const LinComb &c, double *out, hipStream_t s);
/* iterative refinement: r = b - v; x += d */
hipError_t launch_residual(int64_t n, const double *b, const double *v, double *r, hipStream_t s);
hipError_t launch_add_correction(int64_t n, double *x, const float *d, hipStream_t s);
/* kind 0: dst = src (n doubles); kind 1: dst[b] = block partial sums of src */
hipError_t launch_stream(int kind, int64_t n, const double *src, double *dst, int nblocks, hipStream_t s);

/* Comparison solvers (unfused).  Their reductions write per-block records
 * of 8 doubles into a.dots, at most MAX_VEC_BLOCKS of them. */
constexpr int MAX_VEC_BLOCKS = 2048;
int vec_blocks(int64_t n);
/* Algorithm 5 in three passes: pre (r, p, x) ... mat-vec ... post (7 dots) + finish;
 * prec = false: M = I (Algorithm 4), a.dinv not read */
hipError_t launch_alg5_pre(const IterArgs<double> &a, int64_t n, bool prec, hipStream_t s);
hipError_t launch_alg5_post(const IterArgs<double> &a, int64_t n, bool prec, hipStream_t s);
/* Algorithm 1: r^T D^{-1} r -> beta, p = D^{-1} r + beta p ... mat-vec ... p^T v -> alpha, x and r update, ||r||;
 * prec = false: z = r */
hipError_t launch_pcg_direction(const IterArgs<double> &a, int64_t n, bool prec, hipStream_t s);
hipError_t launch_pcg_update(const IterArgs<double> &a, int64_t n, hipStream_t s);

/* Pipelined CG (Algorithm 2), unpreconditioned.  q = A w comes from the
 * operator's mat-vec mode; one fused vector kernel does the six updates and
 * the two inner products, a one-block finish the scalars. */
struct PipeArgs {
    double *x, *r, *p, *w, *s, *z;
    const double *q;
    double *part; /* per-block records of 8 doubles, at most MAX_VEC_BLOCKS */
    CGState *st;
    KrylovState *ks;
    double *hist;
    int64_t n;
};
/* p = s = z = 0, gamma_0 = r^T r, a_0 = w^T r, alpha_1 = gamma_0 / a_0 */
hipError_t launch_pipe_init(const PipeArgs &a, hipStream_t s);
/* the vector updates of one iteration, its inner products and the next scalars */
hipError_t launch_pipe_step(const PipeArgs &a, hipStream_t s);
/* at exit: the step still owed to x after an odd iteration count */
hipError_t launch_pipe_exit(const PipeArgs &a, hipStream_t s);

/* s-step CG (Algorithm 3, monomial basis), unpreconditioned.  T[0] = r and
 * T[1..s] = A^j r (filled by the caller's mat-vecs), P[0..s) the direction
 * block, b the right-hand side and v = A x (internal order). */
constexpr int SSTEP_REC = 80; /* doubles per block record, >= s^2 + s */
struct SStepArgs {
    double *T[SSTEP_MAX + 1];
    double *P[SSTEP_MAX];
    double *x;
    const double *b, *v;
    double *part; /* per-block records of SSTEP_REC doubles, at most MAX_VEC_BLOCKS */
    CGState *st;
    KrylovState *ks;
    double *hist;
    int64_t n;
};
/* C = P_prev^T Q, B = -W_prev^{-1} C; P = R + P_prev B, W = Q^T P, g = P^T r, a = W^{-1} g; x += P a */
hipError_t launch_sstep_blocks(const SStepArgs &a, int sdim, hipStream_t s);
/* r = T[0] = b - v, ||r||, history, convergence test, next phase */
hipError_t launch_sstep_residual(const SStepArgs &a, int sdim, hipStream_t s);

}  // namespace mfcg
