/*
 * mfcg_internal.h -- data structures shared by the host setup code and the
 * gfx950 kernels of the fused CG library.
 *
 * Enumeration of unknowns (the GPU form of Sec. 5.3 of the paper).  The
 * cells are grouped into tiles of TX x TY x TZ cells; one workgroup owns a
 * tile and streams through its cell layers along z.  Per direction the node
 * lattice 0..N*k splits into tile-boundary planes (one node) and the open
 * segments between them; a 3D "entity" is a product of three such 1D
 * pieces, so a tile touches 3^3 = 27 entities (the paper's 3^3 compressed
 * indices per cell, here per tile).  Entities are stored contiguously, x
 * fastest, in the order
 *     [tile interiors (class I) in tile order]
 *     [faces][edges][vertices]          (class S: shared by 2, 4, 8 tiles)
 *     [Dirichlet entities]              (class C: identity rows)
 * so that a tile's interior nodes -- the large majority -- are one
 * contiguous block, read and written once per iteration by one workgroup.
 * Shared nodes receive per-tile partial sums of A p in `partials`
 * (faces: 2 slots, edges: 4, vertices: 8); a second kernel adds them in a
 * fixed order and applies the vector updates and inner products there.
 */
#pragma once
#include <stdint.h>

namespace mfcg {

constexpr int MAXN = 9;  /* k + 1 for k <= 8 */

enum Kind : int32_t { KIND_I = 0, KIND_S = 1, KIND_C = 2 };
enum Flag : int32_t { FLAG_RUN = 0, FLAG_CONV = 1, FLAG_BREAK = 2 };

/* 1D tables in the reference interval [0,1].
 *  S[q*n+i]  = phi_i(xq_q)   GLL-node Lagrange basis at the Gauss points
 *  D[q*n+m]  = l_m'(xq_q)    derivative of the Gauss-point Lagrange basis
 *                            (collocation derivative at quadrature points)
 *  Sd[q*n+i] = phi_i'(xq_q)  = (D S)[q][i]                                */
template <typename T>
struct Tables {
    T S[MAXN * MAXN];
    T D[MAXN * MAXN];
    T Sd[MAXN * MAXN];
    T xq[MAXN];
    T wq[MAXN];
    T gll[MAXN];
};

/* Tile partition of one direction: tile j covers cells
 * [j*T, min((j+1)*T, ncells)). */
struct Dim1 {
    int32_t ncells, T, ntiles, K;
};

/* One of the 27 entities of a tile. */
struct EntityRef {
    int64_t vbase;  /* first node of the entity in the internal vector */
    int64_t pbase;  /* KIND_S: where this tile's partial sums for the entity start */
    int32_t kind;   /* KIND_I / KIND_S / KIND_C */
    int32_t pad;
};

struct TileDesc {
    int32_t c0[3];   /* first cell */
    int32_t nc[3];   /* cells per direction (ragged at the domain end) */
    int64_t gbase;   /* offset of the tile's geometry tensor block (in elements) */
};

/* Device-side view of the enumeration (global memory tables). */
struct LayoutView {
    Dim1 d[3];
    int64_t n;                      /* all nodes */
    int64_t nI, nF, nE, nV, nC;     /* class sizes */
    int64_t offF, offE, offV, offC; /* first node of each class */
    int64_t partF, partE, partV;    /* first element of each class in partials */
    int64_t ntiles;
    const int64_t *ent_base;        /* per 3D entity (ex + ne0*(ey + ne1*ez)) */
    const EntityRef *tile_ent;      /* ntiles * 27 */
    const TileDesc *tiles;          /* ntiles */
};

/* Scalars of Algorithm 5 kept in device memory between launches. */
struct CGState {
    double alpha;    /* alpha_k of the last completed iteration k */
    double beta;     /* beta_k */
    double ratio;    /* alpha_{k-1} / beta_{k-1} */
    double xa;       /* x reconstruction at exit: x += xa p (+ xratio (p - D^{-1} r) if k even) */
    double xratio;
    double eps;      /* tol * ||b|| */
    double bnorm;
    double r0norm;
    int32_t k;       /* completed iterations */
    int32_t flag;    /* FLAG_* */
    int32_t maxit;
    double rz;       /* r^T D^{-1} r of the basic PCG (Algorithm 1) */
};

/* Scalars of the comparison solvers of Sec. 4.1 kept in device memory. */
constexpr int SSTEP_MAX = 8;
struct KrylovState {
    /* pipelined CG (Algorithm 2): the next iteration's alpha and beta and the
     * gamma_k = r^T r, a_k = w^T r they were formed from */
    double alpha, beta, gamma, a;
    /* x is updated every other iteration (two steps at once): alpha_x is
     * the alpha of the last completed iteration, alpha_prev the one before;
     * xpend = 1 while the last iteration's step is still owed to x */
    double alpha_x, alpha_prev;
    int32_t xpend, pad_;
    /* s-step CG (Algorithm 3): completed phases, W = Q^T P of the last phase,
     * the block B and the coefficient vector a of the current phase
     * (row-major s x s) */
    int32_t phase, s;
    double W[SSTEP_MAX * SSTEP_MAX];
    double B[SSTEP_MAX * SSTEP_MAX];
    double avec[SSTEP_MAX];
};

}  // namespace mfcg
