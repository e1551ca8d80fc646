/* kernels.h -- launch wrappers of the gfx950 kernels (host callable). */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mfcg_internal.h"

namespace mfcg {

enum Mode : int { MODE_CG = 0, MODE_VMULT = 1 };

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

/* Maximum tile extent in x and y (cells) compiled for degree K. */
void tile_limits(int K, int *tx, int *ty);
int fused_block_size(int K);

template <typename T>
hipError_t launch_fused(int K, int mode, const IterArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_shared(int mode, const IterArgs<T> &a, hipStream_t s);

/* Setup kernels (FP64). */
struct GeomArgs {
    LayoutView L;
    Tables<double> tab;
    int32_t K, map_kind;
    double amp;
    int32_t bc;
    const double *coeff; /* per cell, device */
};
hipError_t launch_geometry(const GeomArgs &g, double *G, hipStream_t s);
hipError_t launch_diagonal(const GeomArgs &g, const double *G, double *diag_lex, double *dinv_int, hipStream_t s);
hipError_t launch_rhs(const GeomArgs &g, int kind, const double *params, int nparams, double *b_lex, hipStream_t s);

/* Vector utilities. */
template <typename T>
hipError_t launch_lex_to_int(const LayoutView &L, const double *in_lex, T *out_int, hipStream_t s);
template <typename T>
hipError_t launch_int_to_lex(const LayoutView &L, const T *in_int, double *out_lex, hipStream_t s);
/* r = r - v (use_v), p = 0, v = 0 */
hipError_t launch_init_cg(int64_t n, double *r, double *p, double *v, int use_v, hipStream_t s);
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
/* iterative refinement: r = b - v; x += d */
hipError_t launch_residual(int64_t n, const double *b, const double *v, double *r, hipStream_t s);
hipError_t launch_add_correction(int64_t n, double *x, const float *d, hipStream_t s);
/* kind 0: dst = src (n doubles); kind 1: dst[b] = block partial sums of src */
hipError_t launch_stream(int kind, int64_t n, const double *src, double *dst, int nblocks, hipStream_t s);

/* Comparison solvers (unfused).  Their reductions write per-block records
 * of 8 doubles into a.dots, at most MAX_VEC_BLOCKS of them. */
constexpr int MAX_VEC_BLOCKS = 2048;
int vec_blocks(int64_t n);
/* Algorithm 5 in three passes: pre (r, p, x) ... mat-vec ... post (7 dots) + finish */
hipError_t launch_alg5_pre(const IterArgs<double> &a, int64_t n, hipStream_t s);
hipError_t launch_alg5_post(const IterArgs<double> &a, int64_t n, hipStream_t s);
/* Algorithm 1: r^T D^{-1} r -> beta, p = D^{-1} r + beta p ... mat-vec ... p^T v -> alpha, x and r update, ||r|| */
hipError_t launch_pcg_direction(const IterArgs<double> &a, int64_t n, hipStream_t s);
hipError_t launch_pcg_update(const IterArgs<double> &a, int64_t n, hipStream_t s);

}  // namespace mfcg
