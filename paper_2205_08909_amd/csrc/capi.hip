/*
 * capi.hip -- the C-ABI of include/mfcg.h: handle set-up, operator
 * application, the solve driver and the stepping/timing interface.
 *
 * The solve keeps all scalars of Algorithm 5 in device memory; the host
 * only enqueues launches (fused tile kernel + shared-node kernel per
 * iteration) and polls one status word every `check_every` iterations.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mfcg.h"
#include "kernels.h"
#include "setup_host.h"

using namespace mfcg;

struct EventPair {
    hipEvent_t a, b;
};

struct mfcg_ctx {
    int device = 0;
    mfcg_mesh mesh{};
    int K = 0;
    int check_every = 16;
    int solver = MFCG_SOLVER_FUSED;
    int sstep = 6;
    int precond = MFCG_PRECOND_JACOBI;
    bool gll = false; /* quadrature on the GLL nodes (collocation) */
    bool mass = false; /* the mass operator instead of the Laplacian */
    bool q2 = false;   /* k + 2 Gauss points per direction instead of k + 1 */
    bool qgeom = false; /* quadratic geometry evaluated in the operator kernel */
    double *Xq = nullptr; /* its per-cell array (QGEOM_STRIDE doubles per cell) */
    /* solver, preconditioner and s fixed by cg_begin for the solve in progress */
    int solver_active = MFCG_SOLVER_FUSED;
    int sstep_active = 6;
    bool prec_active = true;
    HostLayout hl;
    LayoutView lv{};
    Tables<double> tab{};
    /* device buffers */
    int64_t *d_ent_base = nullptr;
    EntityRef *d_tile_ent = nullptr;
    TileDesc *d_tiles = nullptr;
    double *d_coeff = nullptr;
    double *G = nullptr, *dinv = nullptr, *diag_lex = nullptr;
    double *r = nullptr, *p = nullptr, *v = nullptr, *x = nullptr;
    double *vin = nullptr, *vout = nullptr;
    double *part = nullptr, *dots = nullptr, *sums = nullptr;
    double *hist = nullptr;
    int hist_cap = 0;
    CGState *st = nullptr;
    /* work vectors, block records and scalars of the pipelined and s-step solvers */
    double *kvec = nullptr;
    int64_t kvec_cap = 0; /* vectors of length n */
    double *kpart = nullptr;
    KrylovState *ks = nullptr;
    /* three-component work vectors of the vector Laplacian (component-blocked) */
    double *r3 = nullptr, *p3 = nullptr, *v3 = nullptr, *x3 = nullptr, *dots3 = nullptr, *part3 = nullptr;
    /* work vectors of mfcg_warmstart_span: span_cap vectors each */
    double *spanU = nullptr, *spanAU = nullptr;
    int span_cap = 0;
    /* independent right-hand sides (mfcg_solve_multi): m blocks of each */
    double *rM = nullptr, *pM = nullptr, *vM = nullptr, *xM = nullptr, *dotsM = nullptr, *partM = nullptr;
    double *histM = nullptr;
    CGState *stM = nullptr;
    int mcap = 0;
    int64_t histM_cap = 0;
    int nshared_blocks = 1;
    int nsum_blocks = 1;
    /* solve bookkeeping */
    int maxit = 0;
    int launched = 0;
    double bnorm = 0.0;
    bool zero_rhs = false;
    /* FP32 copy of the operator and FP32 work vectors (iterative refinement) */
    float *G32 = nullptr, *dinv32 = nullptr;
    bool fp32_ready = false; /* the FP32 buffers below are allocated and converted */
    float *r32 = nullptr, *p32 = nullptr, *v32 = nullptr, *x32 = nullptr, *part32 = nullptr, *dots32 = nullptr;
    CGState *st32 = nullptr;
    double *hist32 = nullptr;
    int64_t hist32_cap = 0;
    /* timing */
    bool timing = false;
    std::vector<EventPair> ev_fused, ev_shared, ev_pool;
    std::string err;
};

static thread_local std::string g_last_error;

static int fail(mfcg_ctx *h, int code, const std::string &msg)
{
    if (h)
        h->err = msg;
    else
        g_last_error = msg;
    return code;
}

/* A failed HIP call is reported through the return code; the runtime's
 * last-error state it set is cleared, so that a caller's next HIP call (a
 * framework's allocation, say) is not taken to have failed. */
#define HIPCHK(h, call)                                                                               \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) {                                                                       \
            (void)hipGetLastError();                                                                  \
            return fail((h), e_ == hipErrorOutOfMemory ? MFCG_ENOMEM : MFCG_EHIP,                     \
                        std::string(#call) + ": " + hipGetErrorString(e_));                            \
        }                                                                                             \
    } while (0)

template <typename T>
static hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, sizeof(T) * count);
}

static void release(mfcg_ctx *h)
{
    void *bufs[] = {h->d_ent_base, h->d_tile_ent, h->d_tiles, h->d_coeff, h->G,     h->dinv,   h->diag_lex,
                    h->r,          h->p,          h->v,       h->x,       h->vin,   h->vout,   h->part,
                    h->dots,       h->sums,       h->hist,    h->st,      h->G32,   h->dinv32, h->r32,
                    h->p32,        h->v32,        h->x32,     h->part32,  h->dots32, h->st32,  h->hist32,
                    h->kvec,       h->kpart,      h->ks,      h->r3,      h->p3,    h->v3,     h->x3,
                    h->dots3,      h->part3,      h->Xq,      h->rM,      h->pM,    h->vM,     h->xM,
                    h->dotsM,      h->partM,      h->histM,   h->stM,     h->spanU, h->spanAU};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (auto &e : h->ev_pool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto &e : h->ev_fused) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto &e : h->ev_shared) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
}

static int validate_mesh(const mfcg_mesh *mesh, int32_t degree, const int32_t *tile, std::string &msg)
{
    if (!mesh) {
        msg = "mesh is NULL";
        return MFCG_EINVAL;
    }
    if (degree < 1 || degree > 8) {
        msg = "degree must be in 1..8";
        return MFCG_EINVAL;
    }
    for (int d = 0; d < 3; ++d)
        if (mesh->cells[d] < 1 || mesh->cells[d] > (1 << 20)) {
            msg = "cells must be >= 1";
            return MFCG_EINVAL;
        }
    if (mesh->map_kind < 0 || mesh->map_kind > 2) {
        msg = "unknown map_kind";
        return MFCG_EINVAL;
    }
    if (!std::isfinite(mesh->map_amplitude)) {
        msg = "map amplitude not finite";
        return MFCG_EINVAL;
    }
    if (mesh->bc != MFCG_BC_DIRICHLET0 && mesh->bc != MFCG_BC_NONE) {
        msg = "unknown bc";
        return MFCG_EINVAL;
    }
    int tx, ty;
    tile_limits(degree, &tx, &ty);
    if (tile) {
        for (int d = 0; d < 3; ++d)
            if (tile[d] < 0) {
                msg = "tile sizes must be >= 0";
                return MFCG_EINVAL;
            }
        if (tile[0] > tx || tile[1] > ty) {
            msg = "tile x/y extent exceeds the compiled maximum for this degree";
            return MFCG_EINVAL;
        }
    }
    /* the fused kernels index vectors and partial-sum arrays with 32-bit
     * offsets: at most 2^31 - 1 nodes (the largest stored-tensor problem
     * that fits in 288 GB at Q4 has about 1.8e9) */
    int64_t lat = 1;
    for (int d = 0; d < 3; ++d) lat *= (int64_t)mesh->cells[d] * degree + 1;
    if (lat >= ((int64_t)1 << 31)) {
        msg = "mesh too large: at most 2^31 - 1 nodes";
        return MFCG_EINVAL;
    }
    return MFCG_OK;
}

/* vmult on internal vectors: dst = A src */
/* operator-variant flags for launch_fused */
static int op_flags(const mfcg_ctx *h)
{
    return (h->gll ? MODE_GLL : 0) | (h->mass ? MODE_MASS : 0) | (h->q2 ? MODE_Q2 : 0) | (h->qgeom ? MODE_QGEOM : 0);
}
/* what the operator kernels read as geometry: the stored tensor, or the
 * per-cell quadratic geometry */
static const double *op_geometry(const mfcg_ctx *h) { return h->qgeom ? h->Xq : h->G; }
static int n_q(const mfcg_ctx *h) { return h->K + (h->q2 ? 2 : 1); }

static int vmult_internal(mfcg_ctx *h, const double *src, double *dst, hipStream_t s)
{
    IterArgs<double> a{};
    a.L = h->lv;
    a.G = op_geometry(h);
    a.dinv = h->dinv;
    a.src = src;
    a.dst = dst;
    a.part = h->part;
    a.dots = h->dots;
    a.st = h->st;
    a.hist = h->hist;
    a.nshared_blocks = h->nshared_blocks;
    HIPCHK(h, launch_fused<double>(h->K, MODE_VMULT | op_flags(h), a, s));
    HIPCHK(h, launch_shared<double>(MODE_VMULT, a, s));
    return MFCG_OK;
}

static int ensure_fp32(mfcg_ctx *h, hipStream_t s);

static int host_sumsq(mfcg_ctx *h, const double *a, const double *c, int64_t n, double *out, hipStream_t s)
{
    HIPCHK(h, launch_sumsq(n, a, c, h->sums, h->nsum_blocks, s));
    std::vector<double> tmp(h->nsum_blocks);
    HIPCHK(h, hipMemcpyAsync(tmp.data(), h->sums, sizeof(double) * h->nsum_blocks, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : tmp) t += v;
    *out = t;
    return MFCG_OK;
}

/* fixed-order host sum of the per-block partials of launch_pair_sum */
static int host_pair_sum(mfcg_ctx *h, int mode, const double *a, const double *b, double sc, double *out,
                         hipStream_t s)
{
    HIPCHK(h, launch_pair_sum(h->hl.n, mode, a, b, sc, h->sums, h->nsum_blocks, s));
    std::vector<double> tmp(h->nsum_blocks);
    HIPCHK(h, hipMemcpyAsync(tmp.data(), h->sums, sizeof(double) * h->nsum_blocks, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : tmp) t += v;
    *out = t;
    return MFCG_OK;
}

/* G and the diagonal from the current coefficient; the FP32 copy follows */
static int rebuild_operator(mfcg_ctx *h, hipStream_t s)
{
    GeomArgs g{};
    g.L = h->lv;
    g.tab = h->tab;
    g.K = h->K;
    g.map_kind = h->mesh.map_kind;
    g.amp = h->mesh.map_kind == MFCG_MAP_AFFINE ? 0.0 : h->mesh.map_amplitude;
    g.bc = h->mesh.bc;
    g.coeff = h->d_coeff;
    g.op = h->mass ? 1 : 0;
    g.nq = n_q(h);
    if (h->qgeom) {
        HIPCHK(h, launch_qgeom_nodes(g, h->Xq, s));
        g.X = h->Xq; /* the stored tensor (read by the diagonal) from the same interpolant */
    }
    HIPCHK(h, launch_geometry(g, h->G, s));
    HIPCHK(h, launch_diagonal(g, h->G, h->diag_lex, h->dinv, s));
    if (h->fp32_ready) {
        HIPCHK(h, launch_convert(h->hl.g_elems, h->G, h->G32, s));
        HIPCHK(h, launch_convert(h->hl.n, h->dinv, h->dinv32, s));
    }
    return MFCG_OK;
}

extern "C" {

const char *mfcg_error_string(int code)
{
    switch (code) {
    case MFCG_OK: return "ok";
    case MFCG_EINVAL: return "invalid argument";
    case MFCG_ENOMEM: return "out of device memory";
    case MFCG_EHIP: return "HIP runtime error";
    case MFCG_ENOTCONV: return "not converged within maxit";
    case MFCG_EBREAKDOWN: return "CG breakdown (p^T A p <= 0 or non-finite)";
    case MFCG_ESTAGNATION: return "iterative refinement stagnated";
    default: return "unknown error";
    }
}

const char *mfcg_last_error(mfcg_handle h)
{
    return h ? h->err.c_str() : g_last_error.c_str();
}

int mfcg_layout_permutation(const mfcg_mesh *mesh, int32_t degree, const int32_t *tile, int64_t *perm,
                            int64_t *n_interior, int64_t *n_shared, int64_t *n_dirichlet)
{
    std::string msg;
    int rc = validate_mesh(mesh, degree, tile, msg);
    if (rc) return fail(nullptr, rc, msg);
    HostLayout L;
    int nc[3] = {mesh->cells[0], mesh->cells[1], mesh->cells[2]};
    int t[3] = {tile ? tile[0] : 0, tile ? tile[1] : 0, tile ? tile[2] : 0};
    build_layout(nc, degree, t, mesh->bc, L);
    if (perm) host_permutation(L, perm);
    if (n_interior) *n_interior = L.nI;
    if (n_shared) *n_shared = L.nF + L.nE + L.nV;
    if (n_dirichlet) *n_dirichlet = L.nC;
    return MFCG_OK;
}

int mfcg_setup(const mfcg_mesh *mesh, int32_t degree, const double *cell_coeff, const mfcg_options *opt,
               void *hip_stream, mfcg_handle *out)
{
    if (!out) return fail(nullptr, MFCG_EINVAL, "out is NULL");
    *out = nullptr;
    std::string msg;
    const int32_t *tile = opt ? opt->tile : nullptr;
    int rc = validate_mesh(mesh, degree, tile, msg);
    if (rc) return fail(nullptr, rc, msg);
    if (opt && opt->n_q_1d != 0 && opt->n_q_1d != degree + 1 && opt->n_q_1d != degree + 2)
        return fail(nullptr, MFCG_EINVAL, "n_q_1d must be k+1 or k+2");
    const bool q2 = opt && opt->n_q_1d == degree + 2;
    if (q2 && (degree > 7 || opt->quad_rule != MFCG_QUAD_GAUSS || opt->fp32))
        return fail(nullptr, MFCG_EINVAL, "n_q_1d = k+2: Gauss points, FP64, k <= 7 only");
    if (opt && opt->geometry != MFCG_GEOM_STORED && opt->geometry != MFCG_GEOM_QUADRATIC)
        return fail(nullptr, MFCG_EINVAL, "unknown geometry");
    const bool qgeom = opt && opt->geometry == MFCG_GEOM_QUADRATIC;
    if (qgeom && (opt->quad_rule != MFCG_QUAD_GAUSS || opt->fp32))
        return fail(nullptr, MFCG_EINVAL, "quadratic geometry: Gauss points, FP64 only");
    if (opt && opt->check_every < 0) return fail(nullptr, MFCG_EINVAL, "check_every must be >= 0");
    if (opt && opt->quad_rule != MFCG_QUAD_GAUSS && opt->quad_rule != MFCG_QUAD_GLL)
        return fail(nullptr, MFCG_EINVAL, "unknown quad_rule");
    if (opt && opt->quad_rule == MFCG_QUAD_GLL && opt->fp32)
        return fail(nullptr, MFCG_EINVAL, "the FP32 operator is built for Gauss quadrature only");
    if (opt && opt->op != MFCG_OP_LAPLACE && opt->op != MFCG_OP_MASS)
        return fail(nullptr, MFCG_EINVAL, "unknown operator");
    if (opt && opt->op == MFCG_OP_MASS && (opt->quad_rule != MFCG_QUAD_GAUSS || opt->fp32))
        return fail(nullptr, MFCG_EINVAL, "the mass operator runs in FP64 on the Gauss points only");
    const int64_t ncell = (int64_t)mesh->cells[0] * mesh->cells[1] * mesh->cells[2];
    if (cell_coeff) {
        for (int64_t c = 0; c < ncell; ++c)
            if (!(cell_coeff[c] > 0.0) || !std::isfinite(cell_coeff[c]))
                return fail(nullptr, MFCG_EINVAL, "cell coefficients must be positive and finite");
    }

    mfcg_ctx *h = new (std::nothrow) mfcg_ctx();
    if (!h) return fail(nullptr, MFCG_ENOMEM, "host allocation failed");
    h->mesh = *mesh;
    h->K = degree;
    if (opt && opt->check_every > 0) h->check_every = opt->check_every;
    h->gll = opt && opt->quad_rule == MFCG_QUAD_GLL;
    h->mass = opt && opt->op == MFCG_OP_MASS;
    h->q2 = q2;
    h->qgeom = qgeom;
    hipStream_t s = (hipStream_t)hip_stream;

    auto bail = [&](int code) {
        g_last_error = h->err;
        release(h);
        delete h;
        return code;
    };
#define SCHK(call)                                                                               \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            h->err = std::string(#call) + ": " + hipGetErrorString(e_);                          \
            return bail(e_ == hipErrorOutOfMemory ? MFCG_ENOMEM : MFCG_EHIP);                    \
        }                                                                                        \
    } while (0)

    int nc[3] = {mesh->cells[0], mesh->cells[1], mesh->cells[2]};
    int t[3] = {tile ? tile[0] : 0, tile ? tile[1] : 0, tile ? tile[2] : 0};
    build_layout(nc, degree, t, mesh->bc, h->hl, n_q(h));
    if (h->hl.npart >= ((int64_t)1 << 31)) {
        h->err = "mesh too large: the shared-node partial sums exceed 2^31 - 1 entries";
        return bail(MFCG_EINVAL);
    }
    SCHK(hipGetDevice(&h->device));
    if (build_tables(degree, h->tab, h->gll, n_q(h))) {
        h->err = "quadrature tables";
        return bail(MFCG_EINVAL);
    }
    HostLayout &L = h->hl;

    SCHK(dalloc(&h->d_ent_base, L.ent_base.size()));
    SCHK(dalloc(&h->d_tile_ent, L.tile_ent.size()));
    SCHK(dalloc(&h->d_tiles, L.tiles.size()));
    SCHK(hipMemcpyAsync(h->d_ent_base, L.ent_base.data(), sizeof(int64_t) * L.ent_base.size(),
                        hipMemcpyHostToDevice, s));
    SCHK(hipMemcpyAsync(h->d_tile_ent, L.tile_ent.data(), sizeof(EntityRef) * L.tile_ent.size(),
                        hipMemcpyHostToDevice, s));
    SCHK(hipMemcpyAsync(h->d_tiles, L.tiles.data(), sizeof(TileDesc) * L.tiles.size(), hipMemcpyHostToDevice, s));
    if (cell_coeff) {
        SCHK(dalloc(&h->d_coeff, ncell));
        SCHK(hipMemcpyAsync(h->d_coeff, cell_coeff, sizeof(double) * ncell, hipMemcpyHostToDevice, s));
    }

    LayoutView &lv = h->lv;
    for (int d = 0; d < 3; ++d) lv.d[d] = L.d[d];
    lv.n = L.n;
    lv.nI = L.nI;
    lv.nF = L.nF;
    lv.nE = L.nE;
    lv.nV = L.nV;
    lv.nC = L.nC;
    lv.offF = L.offF;
    lv.offE = L.offE;
    lv.offV = L.offV;
    lv.offC = L.offC;
    lv.partF = L.partF;
    lv.partE = L.partE;
    lv.partV = L.partV;
    lv.ntiles = L.ntiles;
    lv.ent_base = h->d_ent_base;
    lv.tile_ent = h->d_tile_ent;
    lv.tiles = h->d_tiles;

    const int64_t nS = L.n - L.offF;
    h->nshared_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nS + 4 * 256 - 1) / (4 * 256)));
    h->nsum_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (L.n + 1023) / 1024));

    SCHK(dalloc(&h->G, L.g_elems));
    if (h->qgeom) SCHK(dalloc(&h->Xq, ncell * QGEOM_STRIDE));
    SCHK(dalloc(&h->dinv, L.n));
    SCHK(dalloc(&h->diag_lex, L.n));
    SCHK(dalloc(&h->r, L.n));
    SCHK(dalloc(&h->p, L.n));
    SCHK(dalloc(&h->v, L.n));
    SCHK(dalloc(&h->x, L.n));
    SCHK(dalloc(&h->vin, L.n));
    SCHK(dalloc(&h->vout, L.n));
    SCHK(dalloc(&h->part, L.npart));
    /* per-block inner-product records of the fused path, or of the comparison solvers' vector kernels */
    SCHK(dalloc(&h->dots, 8 * std::max<int64_t>(L.ntiles + h->nshared_blocks, MAX_VEC_BLOCKS)));
    SCHK(dalloc(&h->sums, h->nsum_blocks));
    SCHK(dalloc(&h->st, 1));
    h->hist_cap = 1024;
    SCHK(dalloc(&h->hist, h->hist_cap + 1));
    /* slots of shared nodes that no tile owns (domain boundary without
     * Dirichlet condition) must read as zero */
    SCHK(hipMemsetAsync(h->part, 0, sizeof(double) * std::max<int64_t>(1, L.npart), s));
    SCHK(hipMemsetAsync(h->st, 0, sizeof(CGState), s));

    if (rebuild_operator(h, s)) return bail(MFCG_EHIP);
    if (opt && opt->fp32) {
        if (ensure_fp32(h, s)) return bail(MFCG_EHIP);
    }
    SCHK(hipStreamSynchronize(s));
#undef SCHK
    *out = h;
    return MFCG_OK;
}

int mfcg_set_coefficient(mfcg_handle h, const double *cell_coeff, void *hip_stream)
{
    if (!h) return fail(h, MFCG_EINVAL, "null handle");
    const int64_t ncell = (int64_t)h->mesh.cells[0] * h->mesh.cells[1] * h->mesh.cells[2];
    if (cell_coeff) {
        for (int64_t c = 0; c < ncell; ++c)
            if (!(cell_coeff[c] > 0.0) || !std::isfinite(cell_coeff[c]))
                return fail(h, MFCG_EINVAL, "cell coefficients must be positive and finite");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (cell_coeff) {
        if (!h->d_coeff) HIPCHK(h, dalloc(&h->d_coeff, ncell));
        HIPCHK(h, hipMemcpyAsync(h->d_coeff, cell_coeff, sizeof(double) * ncell, hipMemcpyHostToDevice, s));
    } else if (h->d_coeff) {
        HIPCHK(h, hipStreamSynchronize(s));
        HIPCHK(h, hipFree(h->d_coeff));
        h->d_coeff = nullptr;
    }
    int rc = rebuild_operator(h, s);
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(s));
    return MFCG_OK;
}

int mfcg_warmstart(mfcg_handle h, const double *b, const double *u, double max_rel_res, double *x0, double *scale,
                   double *rel_res, int32_t *used, void *hip_stream)
{
    if (!h || !b || !u || !x0) return fail(h, MFCG_EINVAL, "null argument");
    if (std::isnan(max_rel_res)) return fail(h, MFCG_EINVAL, "max_rel_res is NaN");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = h->hl.n;
    /* internal order: p = u with the Dirichlet block zeroed, v = A p, r = b */
    HIPCHK(h, launch_lex_to_int<double>(h->lv, u, h->p, s));
    if (h->lv.nC > 0) HIPCHK(h, hipMemsetAsync(h->p + h->lv.offC, 0, sizeof(double) * h->lv.nC, s));
    int rc = vmult_internal(h, h->p, h->v, s);
    if (rc) return rc;
    HIPCHK(h, launch_lex_to_int<double>(h->lv, b, h->r, s));
    double ub = 0.0, uau = 0.0, bb = 0.0;
    if ((rc = host_pair_sum(h, 0, h->p, h->r, 0.0, &ub, s))) return rc;
    if ((rc = host_pair_sum(h, 0, h->p, h->v, 0.0, &uau, s))) return rc;
    if ((rc = host_pair_sum(h, 0, h->r, h->r, 0.0, &bb, s))) return rc;
    double sc = (uau > 0.0 && std::isfinite(uau) && std::isfinite(ub)) ? ub / uau : 0.0;
    bool ok = sc != 0.0 && std::isfinite(sc);
    double rel = 1.0;
    if (ok) {
        double rr = 0.0; /* ||b - A (sc p)||^2 */
        if ((rc = host_pair_sum(h, 1, h->r, h->v, sc, &rr, s))) return rc;
        rel = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        ok = std::isfinite(rr) && !(rel >= max_rel_res);
    }
    if (ok) {
        HIPCHK(h, launch_scale(n, h->p, sc, h->vout, s));
        HIPCHK(h, launch_int_to_lex<double>(h->lv, h->vout, x0, s));
    } else {
        HIPCHK(h, hipMemsetAsync(x0, 0, sizeof(double) * n, s));
    }
    HIPCHK(h, hipStreamSynchronize(s));
    if (scale) *scale = ok ? sc : 0.0;
    if (rel_res) *rel_res = ok ? rel : 1.0;
    if (used) *used = ok ? 1 : 0;
    return MFCG_OK;
}

int mfcg_interpolate(mfcg_handle from, const double *src, mfcg_handle to, double *dst, void *hip_stream)
{
    if (!from || !to || !src || !dst) return fail(to ? to : from, MFCG_EINVAL, "null argument");
    for (int d = 0; d < 3; ++d)
        if (from->mesh.cells[d] != to->mesh.cells[d])
            return fail(to, MFCG_EINVAL, "interpolation needs the same cells on both handles");
    if (src == dst) return fail(to, MFCG_EINVAL, "src and dst must differ");
    InterpArgs ia{};
    for (int d = 0; d < 3; ++d) ia.ncells[d] = to->mesh.cells[d];
    ia.kf = from->K;
    ia.kt = to->K;
    interp_weights(ia.kf, ia.kt, ia.W);
    ia.src = src;
    ia.dst = dst;
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(to, launch_interpolate(ia, s));
    HIPCHK(to, hipStreamSynchronize(s));
    return MFCG_OK;
}

int mfcg_warmstart_span(mfcg_handle h, const double *b, int32_t m, const double *const *u, double max_rel_res,
                        double *x0, double *coef, double *rel_res, int32_t *used, void *hip_stream)
{
    if (!h || !b || !u || !x0) return fail(h, MFCG_EINVAL, "null argument");
    if (m < 1 || m > MFCG_SPAN_MAX) return fail(h, MFCG_EINVAL, "m must be in 1..MFCG_SPAN_MAX");
    for (int i = 0; i < m; ++i)
        if (!u[i]) return fail(h, MFCG_EINVAL, "null vector u[" + std::to_string(i) + "]");
    if (std::isnan(max_rel_res)) return fail(h, MFCG_EINVAL, "max_rel_res is NaN");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = h->hl.n;
    if (m > h->span_cap) {
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->spanU) HIPCHK(h, hipFree(h->spanU));
        if (h->spanAU) HIPCHK(h, hipFree(h->spanAU));
        h->spanU = h->spanAU = nullptr;
        h->span_cap = 0;
        HIPCHK(h, dalloc(&h->spanU, (size_t)(m * n)));
        HIPCHK(h, dalloc(&h->spanAU, (size_t)(m * n)));
        h->span_cap = m;
    }
    /* internal order: U_i = u_i with the Dirichlet block zeroed, AU_i = A U_i, r = b */
    for (int i = 0; i < m; ++i) {
        double *Ui = h->spanU + i * n;
        HIPCHK(h, launch_lex_to_int<double>(h->lv, u[i], Ui, s));
        if (h->lv.nC > 0) HIPCHK(h, hipMemsetAsync(Ui + h->lv.offC, 0, sizeof(double) * h->lv.nC, s));
        int rc = vmult_internal(h, Ui, h->spanAU + i * n, s);
        if (rc) return rc;
    }
    HIPCHK(h, launch_lex_to_int<double>(h->lv, b, h->r, s));
    /* Gram system G c = g, G_ij = U_i^T A U_j, g_i = U_i^T b (fixed-order sums) */
    double G[MFCG_SPAN_MAX][MFCG_SPAN_MAX], g[MFCG_SPAN_MAX], bb = 0.0;
    int rc;
    for (int i = 0; i < m; ++i) {
        for (int j = i; j < m; ++j) {
            if ((rc = host_pair_sum(h, 0, h->spanU + i * n, h->spanAU + j * n, 0.0, &G[i][j], s))) return rc;
            G[j][i] = G[i][j];
        }
        if ((rc = host_pair_sum(h, 0, h->spanU + i * n, h->r, 0.0, &g[i], s))) return rc;
    }
    if ((rc = host_pair_sum(h, 0, h->r, h->r, 0.0, &bb, s))) return rc;
    /* Cholesky factorisation in order; a direction whose pivot is not above
     * 1e-12 of its own A-norm square (zero, or in the span of the earlier
     * ones) is dropped (coefficient 0) */
    double L[MFCG_SPAN_MAX][MFCG_SPAN_MAX] = {}, c[MFCG_SPAN_MAX] = {}, y[MFCG_SPAN_MAX] = {};
    bool keep[MFCG_SPAN_MAX] = {};
    bool ok = std::isfinite(bb);
    for (int i = 0; i < m && ok; ++i) {
        double d = G[i][i];
        for (int k = 0; k < i; ++k)
            if (keep[k]) d -= L[i][k] * L[i][k];
        keep[i] = std::isfinite(d) && std::isfinite(G[i][i]) && G[i][i] > 0.0 && d > 1e-12 * G[i][i];
        if (!keep[i]) continue;
        L[i][i] = std::sqrt(d);
        for (int j = i + 1; j < m; ++j) {
            double t = G[j][i];
            for (int k = 0; k < i; ++k)
                if (keep[k]) t -= L[j][k] * L[i][k];
            L[j][i] = t / L[i][i];
        }
    }
    int nkeep = 0;
    for (int i = 0; i < m; ++i) nkeep += keep[i];
    ok = ok && nkeep > 0;
    if (ok) {
        for (int i = 0; i < m; ++i) { /* L y = g */
            if (!keep[i]) continue;
            double t = g[i];
            for (int k = 0; k < i; ++k)
                if (keep[k]) t -= L[i][k] * y[k];
            y[i] = t / L[i][i];
        }
        for (int i = m - 1; i >= 0; --i) { /* L^T c = y */
            if (!keep[i]) continue;
            double t = y[i];
            for (int k = i + 1; k < m; ++k)
                if (keep[k]) t -= L[k][i] * c[k];
            c[i] = t / L[i][i];
        }
        for (int i = 0; i < m; ++i) ok = ok && std::isfinite(c[i]);
    }
    double rel = 1.0;
    if (ok) {
        LinComb lc{};
        for (int i = 0; i < m; ++i) lc.c[i] = c[i];
        HIPCHK(h, launch_lincomb(n, m, h->spanU, lc, h->vout, s));  /* x0 */
        HIPCHK(h, launch_lincomb(n, m, h->spanAU, lc, h->v, s));    /* A x0 */
        double rr = 0.0;
        if ((rc = host_pair_sum(h, 1, h->r, h->v, 1.0, &rr, s))) return rc;
        rel = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        ok = std::isfinite(rr) && !(rel >= max_rel_res);
    }
    if (ok) {
        HIPCHK(h, launch_int_to_lex<double>(h->lv, h->vout, x0, s));
    } else {
        HIPCHK(h, hipMemsetAsync(x0, 0, sizeof(double) * n, s));
    }
    HIPCHK(h, hipStreamSynchronize(s));
    if (coef)
        for (int i = 0; i < m; ++i) coef[i] = ok ? c[i] : 0.0;
    if (rel_res) *rel_res = ok ? rel : 1.0;
    if (used) *used = ok ? 1 : 0;
    return MFCG_OK;
}

int mfcg_destroy(mfcg_handle h)
{
    if (!h) return MFCG_OK;
    (void)hipDeviceSynchronize();
    release(h);
    delete h;
    return MFCG_OK;
}

int mfcg_n_dofs(mfcg_handle h, int64_t *n)
{
    if (!h || !n) return fail(h, MFCG_EINVAL, "null argument");
    *n = h->hl.n;
    return MFCG_OK;
}

int mfcg_layout_info(mfcg_handle h, int32_t *tile, int64_t *n_interior, int64_t *n_shared, int64_t *n_dirichlet,
                     int64_t *n_tiles, int64_t *geometry_bytes)
{
    if (!h) return fail(h, MFCG_EINVAL, "null handle");
    if (tile)
        for (int d = 0; d < 3; ++d) tile[d] = h->hl.d[d].T;
    if (n_interior) *n_interior = h->hl.nI;
    if (n_shared) *n_shared = h->hl.nF + h->hl.nE + h->hl.nV;
    if (n_dirichlet) *n_dirichlet = h->hl.nC;
    if (n_tiles) *n_tiles = h->hl.ntiles;
    if (geometry_bytes) *geometry_bytes = h->hl.g_elems * (int64_t)sizeof(double);
    return MFCG_OK;
}

int mfcg_vmult(mfcg_handle h, double *dst, const double *src, void *hip_stream)
{
    if (!h || !dst || !src) return fail(h, MFCG_EINVAL, "null argument");
    if (dst == src) return fail(h, MFCG_EINVAL, "dst and src must differ");
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(h, launch_lex_to_int<double>(h->lv, src, h->vin, s));
    int rc = vmult_internal(h, h->vin, h->vout, s);
    if (rc) return rc;
    HIPCHK(h, launch_int_to_lex<double>(h->lv, h->vout, dst, s));
    return MFCG_OK;
}

int mfcg_vmult_fp32(mfcg_handle h, double *dst, const double *src, void *hip_stream)
{
    if (!h || !dst || !src) return fail(h, MFCG_EINVAL, "null argument");
    if (dst == src) return fail(h, MFCG_EINVAL, "dst and src must differ");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = ensure_fp32(h, s);
    if (rc) return rc;
    IterArgs<float> a{};
    a.L = h->lv;
    a.G = h->G32;
    a.dinv = h->dinv32;
    a.src = h->r32;
    a.dst = h->v32;
    a.part = h->part32;
    a.dots = h->dots32;
    a.st = h->st32;
    a.nshared_blocks = h->nshared_blocks;
    HIPCHK(h, launch_lex_to_int<float>(h->lv, src, h->r32, s));
    HIPCHK(h, launch_fused<float>(h->K, MODE_VMULT, a, s));
    HIPCHK(h, launch_shared<float>(MODE_VMULT, a, s));
    HIPCHK(h, launch_int_to_lex<float>(h->lv, h->v32, dst, s));
    return MFCG_OK;
}

int mfcg_diagonal(mfcg_handle h, double *diag, void *hip_stream)
{
    if (!h || !diag) return fail(h, MFCG_EINVAL, "null argument");
    HIPCHK(h, hipMemcpyAsync(diag, h->diag_lex, sizeof(double) * h->hl.n, hipMemcpyDeviceToDevice,
                             (hipStream_t)hip_stream));
    return MFCG_OK;
}

int mfcg_assemble_rhs(mfcg_handle h, int32_t kind, const double *params, double *b, void *hip_stream)
{
    if (!h || !b) return fail(h, MFCG_EINVAL, "null argument");
    if (kind != MFCG_RHS_SINE && kind != MFCG_RHS_BUMPS) return fail(h, MFCG_EINVAL, "unknown rhs kind");
    int np = 0;
    if (kind == MFCG_RHS_BUMPS) {
        if (!params) return fail(h, MFCG_EINVAL, "bump parameters missing");
        const int nb = (int)params[0];
        if (!(params[0] >= 0) || nb > 16 || (double)nb != params[0]) return fail(h, MFCG_EINVAL, "bad bump count");
        np = 1 + 5 * nb;
    }
    GeomArgs g{};
    g.L = h->lv;
    g.tab = h->tab;
    g.K = h->K;
    g.map_kind = h->mesh.map_kind;
    g.amp = h->mesh.map_kind == MFCG_MAP_AFFINE ? 0.0 : h->mesh.map_amplitude;
    g.bc = h->mesh.bc;
    g.coeff = h->d_coeff;
    g.nq = n_q(h);
    g.X = h->qgeom ? h->Xq : nullptr;
    HIPCHK(h, launch_rhs(g, kind, params, np, b, (hipStream_t)hip_stream));
    return MFCG_OK;
}

int mfcg_set_timing(mfcg_handle h, int32_t enable)
{
    if (!h) return fail(h, MFCG_EINVAL, "null handle");
    h->timing = enable != 0;
    for (auto &e : h->ev_fused) h->ev_pool.push_back(e);
    for (auto &e : h->ev_shared) h->ev_pool.push_back(e);
    h->ev_fused.clear();
    h->ev_shared.clear();
    return MFCG_OK;
}

static int get_events(mfcg_ctx *h, EventPair &e)
{
    if (!h->ev_pool.empty()) {
        e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return MFCG_OK;
    }
    HIPCHK(h, hipEventCreate(&e.a));
    HIPCHK(h, hipEventCreate(&e.b));
    return MFCG_OK;
}

int mfcg_get_timing(mfcg_handle h, double *fused_ms, int64_t *fused_launches, double *shared_ms,
                    int64_t *shared_launches)
{
    if (!h) return fail(h, MFCG_EINVAL, "null handle");
    double tf = 0.0, ts = 0.0;
    for (auto &e : h->ev_fused) {
        HIPCHK(h, hipEventSynchronize(e.b));
        float ms = 0.0f;
        HIPCHK(h, hipEventElapsedTime(&ms, e.a, e.b));
        tf += ms;
    }
    for (auto &e : h->ev_shared) {
        HIPCHK(h, hipEventSynchronize(e.b));
        float ms = 0.0f;
        HIPCHK(h, hipEventElapsedTime(&ms, e.a, e.b));
        ts += ms;
    }
    if (fused_ms) *fused_ms = tf;
    if (shared_ms) *shared_ms = ts;
    if (fused_launches) *fused_launches = (int64_t)h->ev_fused.size();
    if (shared_launches) *shared_launches = (int64_t)h->ev_shared.size();
    return MFCG_OK;
}

int mfcg_set_solver(mfcg_handle h, int32_t solver)
{
    if (!h) return fail(h, MFCG_EINVAL, "null handle");
    if (solver < MFCG_SOLVER_FUSED || solver > MFCG_SOLVER_SSTEP) return fail(h, MFCG_EINVAL, "unknown solver");
    h->solver = solver;
    return MFCG_OK;
}

int mfcg_set_preconditioner(mfcg_handle h, int32_t precond)
{
    if (!h) return fail(h, MFCG_EINVAL, "null handle");
    if (precond != MFCG_PRECOND_JACOBI && precond != MFCG_PRECOND_NONE)
        return fail(h, MFCG_EINVAL, "unknown preconditioner");
    h->precond = precond;
    return MFCG_OK;
}

int mfcg_set_sstep(mfcg_handle h, int32_t s)
{
    if (!h) return fail(h, MFCG_EINVAL, "null handle");
    if (s < 1 || s > SSTEP_MAX) return fail(h, MFCG_EINVAL, "s must be in 1..8");
    h->sstep = s;
    return MFCG_OK;
}

/* Work space of the pipelined (w, s, z) and s-step (T[1..s], P[0..s), b)
 * solvers, grown on demand. */
static int ensure_krylov(mfcg_ctx *h, int64_t nvec, hipStream_t s)
{
    if (!h->kpart || !h->ks) {
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->kpart) HIPCHK(h, hipFree(h->kpart));
        if (h->ks) HIPCHK(h, hipFree(h->ks));
        h->kpart = nullptr;
        h->ks = nullptr;
        HIPCHK(h, dalloc(&h->kpart, (size_t)MAX_VEC_BLOCKS * SSTEP_REC));
        HIPCHK(h, dalloc(&h->ks, 1));
    }
    if (nvec > h->kvec_cap) {
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->kvec) HIPCHK(h, hipFree(h->kvec));
        h->kvec = nullptr;
        h->kvec_cap = 0;
        HIPCHK(h, dalloc(&h->kvec, (size_t)(nvec * h->hl.n)));
        h->kvec_cap = nvec;
    }
    return MFCG_OK;
}

static PipeArgs pipe_args(mfcg_ctx *h)
{
    const int64_t n = h->hl.n;
    PipeArgs a{};
    a.x = h->x;
    a.r = h->r;
    a.p = h->p;
    a.w = h->kvec;
    a.s = h->kvec + n;
    a.z = h->kvec + 2 * n;
    a.q = h->v;
    a.part = h->kpart;
    a.st = h->st;
    a.ks = h->ks;
    a.hist = h->hist;
    a.n = n;
    return a;
}

static SStepArgs sstep_args(mfcg_ctx *h)
{
    const int64_t n = h->hl.n;
    const int S = h->sstep_active;
    SStepArgs a{};
    a.T[0] = h->r;
    for (int j = 1; j <= S; ++j) a.T[j] = h->kvec + (int64_t)(j - 1) * n;
    for (int m = 0; m < S; ++m) a.P[m] = h->kvec + (int64_t)(S + m) * n;
    a.b = h->kvec + (int64_t)(2 * S) * n;
    a.x = h->x;
    a.v = h->v;
    a.part = h->kpart;
    a.st = h->st;
    a.ks = h->ks;
    a.hist = h->hist;
    a.n = n;
    return a;
}

int mfcg_cg_begin(mfcg_handle h, const double *b, const double *x0, double tol, int32_t maxit, void *hip_stream)
{
    if (!h || !b) return fail(h, MFCG_EINVAL, "null argument");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(h, MFCG_EINVAL, "tol must be finite and >= 0");
    if (maxit < 1) return fail(h, MFCG_EINVAL, "maxit must be >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    if (maxit > h->hist_cap) {
        HIPCHK(h, hipStreamSynchronize(s));
        HIPCHK(h, hipFree(h->hist));
        h->hist = nullptr;
        h->hist_cap = 0; /* a failed allocation leaves no buffer behind */
        HIPCHK(h, dalloc(&h->hist, (size_t)maxit + 1));
        h->hist_cap = maxit;
    }
    const int64_t n = h->hl.n;
    int rc = MFCG_OK;
    if (h->solver == MFCG_SOLVER_PIPELINED) rc = ensure_krylov(h, 3, s);
    if (h->solver == MFCG_SOLVER_SSTEP) rc = ensure_krylov(h, 2 * h->sstep + 1, s);
    if (rc) return rc;
    h->sstep_active = h->sstep;
    h->solver_active = h->solver;
    h->prec_active = h->precond == MFCG_PRECOND_JACOBI;
    /* r = b (internal order); x = x0 or 0 */
    HIPCHK(h, launch_lex_to_int<double>(h->lv, b, h->r, s));
    if (h->solver == MFCG_SOLVER_SSTEP)
        HIPCHK(h, hipMemcpyAsync(h->kvec + (int64_t)(2 * h->sstep) * n, h->r, sizeof(double) * n,
                                 hipMemcpyDeviceToDevice, s));
    double bb = 0.0;
    rc = host_sumsq(h, h->r, nullptr, n, &bb, s);
    if (rc) return rc;
    h->bnorm = std::sqrt(bb);
    h->zero_rhs = (bb == 0.0);
    const bool use_x0 = x0 != nullptr && !h->zero_rhs;
    if (use_x0) {
        HIPCHK(h, launch_lex_to_int<double>(h->lv, x0, h->x, s));
        rc = vmult_internal(h, h->x, h->v, s);
        if (rc) return rc;
    } else {
        HIPCHK(h, hipMemsetAsync(h->x, 0, sizeof(double) * n, s));
    }
    HIPCHK(h, launch_init_cg(n, h->r, h->p, h->v, use_x0 ? 1 : 0, s));
    double rr = 0.0;
    rc = host_sumsq(h, h->r, nullptr, n, &rr, s);
    if (rc) return rc;
    CGState st{};
    st.eps = tol * h->bnorm;
    st.bnorm = h->bnorm;
    st.r0norm = std::sqrt(rr);
    st.maxit = maxit;
    st.flag = (h->zero_rhs || st.r0norm < st.eps) ? FLAG_CONV : FLAG_RUN;
    HIPCHK(h, hipMemcpyAsync(h->st, &st, sizeof(CGState), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->hist, &st.r0norm, sizeof(double), hipMemcpyHostToDevice, s));
    if (h->solver == MFCG_SOLVER_PIPELINED || h->solver == MFCG_SOLVER_SSTEP) {
        KrylovState ks{};
        ks.s = h->sstep;
        HIPCHK(h, hipMemcpyAsync(h->ks, &ks, sizeof(KrylovState), hipMemcpyHostToDevice, s));
    }
    if (h->solver == MFCG_SOLVER_PIPELINED) {
        /* w_0 = A r_0, p = s = z = 0, alpha_1 = gamma_0 / a_0 */
        const PipeArgs pa = pipe_args(h);
        rc = vmult_internal(h, pa.r, pa.w, s);
        if (rc) return rc;
        HIPCHK(h, launch_pipe_init(pa, s));
    }
    h->maxit = maxit;
    h->launched = 0;
    return MFCG_OK;
}

int mfcg_cg_iterate(mfcg_handle h, int32_t n_it, void *hip_stream)
{
    if (!h || n_it < 0) return fail(h, MFCG_EINVAL, "bad argument");
    if (h->launched + n_it > h->maxit) return fail(h, MFCG_EINVAL, "iterations beyond maxit");
    hipStream_t s = (hipStream_t)hip_stream;
    IterArgs<double> a{};
    a.L = h->lv;
    a.G = op_geometry(h);
    a.dinv = h->dinv;
    a.r = h->r;
    a.p = h->p;
    a.v = h->v;
    a.x = h->x;
    a.part = h->part;
    a.dots = h->dots;
    a.st = h->st;
    a.hist = h->hist;
    a.nshared_blocks = h->nshared_blocks;
    const int64_t n = h->hl.n;
    if (h->solver_active == MFCG_SOLVER_PIPELINED) {
        const PipeArgs pa = pipe_args(h);
        for (int it = 0; it < n_it; ++it) {
            int rc = vmult_internal(h, pa.w, h->v, s); /* q = A w */
            if (rc) return rc;
            HIPCHK(h, launch_pipe_step(pa, s));
        }
        h->launched += n_it;
        return MFCG_OK;
    }
    if (h->solver_active == MFCG_SOLVER_SSTEP) {
        /* a phase starts at every multiple of s and runs only if it fits in maxit */
        const int S = h->sstep_active;
        const SStepArgs sa = sstep_args(h);
        for (int it = 0; it < n_it; ++it) {
            const int i = h->launched + it;
            if (i % S != 0 || i + S > h->maxit) continue;
            for (int j = 1; j <= S; ++j) {
                int rc = vmult_internal(h, sa.T[j - 1], sa.T[j], s);
                if (rc) return rc;
            }
            HIPCHK(h, launch_sstep_blocks(sa, S, s));
            int rc = vmult_internal(h, sa.x, h->v, s);
            if (rc) return rc;
            HIPCHK(h, launch_sstep_residual(sa, S, s));
        }
        h->launched += n_it;
        return MFCG_OK;
    }
    for (int it = 0; it < n_it; ++it) {
        if (h->solver_active == MFCG_SOLVER_ALG5_SPLIT) {
            /* pre, mat-vec v = A p, post + finish */
            HIPCHK(h, launch_alg5_pre(a, n, h->prec_active, s));
            IterArgs<double> m = a;
            m.src = h->p;
            m.dst = h->v;
            HIPCHK(h, launch_fused<double>(h->K, MODE_VMULT | op_flags(h), m, s));
            HIPCHK(h, launch_shared<double>(MODE_VMULT, m, s));
            HIPCHK(h, launch_alg5_post(a, n, h->prec_active, s));
            continue;
        }
        if (h->solver_active == MFCG_SOLVER_PCG_BASIC) {
            HIPCHK(h, launch_pcg_direction(a, n, h->prec_active, s));
            IterArgs<double> m = a;
            m.src = h->p;
            m.dst = h->v;
            HIPCHK(h, launch_fused<double>(h->K, MODE_VMULT | op_flags(h), m, s));
            HIPCHK(h, launch_shared<double>(MODE_VMULT, m, s));
            HIPCHK(h, launch_pcg_update(a, n, s));
            continue;
        }
        EventPair e1{}, e2{};
        if (h->timing) {
            int rc = get_events(h, e1);
            if (rc) return rc;
            rc = get_events(h, e2);
            if (rc) return rc;
            HIPCHK(h, hipEventRecord(e1.a, s));
        }
        const int mode = h->prec_active ? MODE_CG : MODE_CG_NOPREC;
        HIPCHK(h, launch_fused<double>(h->K, mode | op_flags(h), a, s));
        if (h->timing) {
            HIPCHK(h, hipEventRecord(e1.b, s));
            HIPCHK(h, hipEventRecord(e2.a, s));
        }
        HIPCHK(h, launch_shared<double>(mode, a, s));
        if (h->timing) {
            HIPCHK(h, hipEventRecord(e2.b, s));
            h->ev_fused.push_back(e1);
            h->ev_shared.push_back(e2);
        }
    }
    h->launched += n_it;
    return MFCG_OK;
}

static int read_state(mfcg_ctx *h, CGState &st, hipStream_t s)
{
    HIPCHK(h, hipMemcpyAsync(&st, h->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return MFCG_OK;
}

int mfcg_cg_end(mfcg_handle h, double *x, int32_t *iters, double *res_hist, void *hip_stream)
{
    if (!h || !x) return fail(h, MFCG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)hip_stream;
    CGState st{};
    int rc = read_state(h, st, s);
    if (rc) return rc;
    if (h->zero_rhs) {
        HIPCHK(h, hipMemsetAsync(x, 0, sizeof(double) * h->hl.n, s));
        if (iters) *iters = 0;
        if (res_hist) res_hist[0] = 0.0;
        HIPCHK(h, hipStreamSynchronize(s));
        return MFCG_OK;
    }
    if (h->solver_active == MFCG_SOLVER_PIPELINED) {
        HIPCHK(h, launch_pipe_exit(pipe_args(h), s));
        HIPCHK(h, hipMemsetAsync(&h->ks->xpend, 0, sizeof(int32_t), s)); /* the step is paid */
    }
    if (h->solver_active == MFCG_SOLVER_FUSED || h->solver_active == MFCG_SOLVER_ALG5_SPLIT) /* Algorithm 5 keeps x behind */
        HIPCHK(h, launch_reconstruct<double>(h->hl.n, h->x, h->p, h->r, h->prec_active ? h->dinv : nullptr,
                                             h->st, s));
    HIPCHK(h, launch_int_to_lex<double>(h->lv, h->x, x, s));
    if (res_hist) HIPCHK(h, hipMemcpyAsync(res_hist, h->hist, sizeof(double) * (st.k + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (iters) *iters = st.k;
    if (st.flag == FLAG_CONV) return MFCG_OK;
    if (st.flag == FLAG_BREAK) return fail(h, MFCG_EBREAKDOWN, "breakdown: p^T A p <= 0 or non-finite scalar");
    return fail(h, MFCG_ENOTCONV, "maxit reached");
}

/* Independent right-hand sides on one operator (Algorithm 5 for each,
 * with its own scalars and stopping test): every iteration runs one fused
 * launch over (tile, right-hand side) pairs, so a tile's geometry tensor is
 * fetched once and served from L2 to the other right-hand sides, then the
 * shared-node kernel over (block, right-hand side) and one finish block per
 * right-hand side.  A right-hand side that has converged or broken down
 * drops out (its workgroups return at once) while the others continue. */
int mfcg_solve_multi(mfcg_handle h, int32_t m, const double *const *b, double *const *x, double tol, int32_t maxit,
                     int32_t *iters, int32_t *status, double *true_rel_res, void *hip_stream)
{
    if (!h || !b || !x || !iters || !status) return fail(h, MFCG_EINVAL, "null argument");
    if (m < 1 || m > MFCG_MULTI_MAX) return fail(h, MFCG_EINVAL, "m must be in 1..MFCG_MULTI_MAX");
    for (int c = 0; c < m; ++c)
        if (!b[c] || !x[c]) return fail(h, MFCG_EINVAL, "null vector of right-hand side " + std::to_string(c));
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(h, MFCG_EINVAL, "tol must be finite and >= 0");
    if (maxit < 1) return fail(h, MFCG_EINVAL, "maxit must be >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = h->hl.n;
    const int64_t nrec = h->hl.ntiles + h->nshared_blocks; /* records per right-hand side */
    const int64_t ps = std::max<int64_t>(1, h->hl.npart);
    /* the device CG state of a scalar solve is not touched, but its work
     * vectors are: a stepping solve in progress ends here */
    h->maxit = 0;
    h->launched = 0;
    if (m > h->mcap) {
        HIPCHK(h, hipStreamSynchronize(s));
        double *bufs[] = {h->rM, h->pM, h->vM, h->xM, h->dotsM, h->partM};
        for (double *q : bufs)
            if (q) HIPCHK(h, hipFree(q));
        if (h->stM) HIPCHK(h, hipFree(h->stM));
        h->rM = h->pM = h->vM = h->xM = h->dotsM = h->partM = nullptr;
        h->stM = nullptr;
        h->mcap = 0;
        HIPCHK(h, dalloc(&h->rM, (size_t)(m * n)));
        HIPCHK(h, dalloc(&h->pM, (size_t)(m * n)));
        HIPCHK(h, dalloc(&h->vM, (size_t)(m * n)));
        HIPCHK(h, dalloc(&h->xM, (size_t)(m * n)));
        HIPCHK(h, dalloc(&h->dotsM, (size_t)(8 * m * nrec)));
        HIPCHK(h, dalloc(&h->partM, (size_t)(m * ps)));
        HIPCHK(h, dalloc(&h->stM, (size_t)m));
        HIPCHK(h, hipMemsetAsync(h->partM, 0, sizeof(double) * m * ps, s));
        h->mcap = m;
    }
    /* history entries per right-hand side, in 64 bits (maxit + 1 overflows
     * 32 bits at maxit = INT32_MAX) */
    const int64_t hs = (int64_t)maxit + 1;
    if ((int64_t)m * hs > h->histM_cap) {
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->histM) HIPCHK(h, hipFree(h->histM));
        h->histM = nullptr;
        h->histM_cap = 0;
        HIPCHK(h, dalloc(&h->histM, (size_t)((int64_t)m * hs)));
        h->histM_cap = (int64_t)m * hs;
    }
    std::vector<CGState> st(m);
    std::vector<char> zero(m, 0);
    for (int c = 0; c < m; ++c) {
        double *rc_ = h->rM + c * n, *pc = h->pM + c * n, *vc = h->vM + c * n, *xc = h->xM + c * n;
        HIPCHK(h, launch_lex_to_int<double>(h->lv, b[c], rc_, s));
        double bb = 0.0;
        int rc = host_sumsq(h, rc_, nullptr, n, &bb, s);
        if (rc) return rc;
        st[c] = CGState{};
        st[c].maxit = maxit;
        if (bb == 0.0) { /* x = 0 exactly, no iteration */
            zero[c] = 1;
            st[c].flag = FLAG_CONV;
            HIPCHK(h, hipMemcpyAsync(h->histM + c * hs, &st[c].r0norm, sizeof(double), hipMemcpyHostToDevice, s));
            continue;
        }
        HIPCHK(h, launch_lex_to_int<double>(h->lv, x[c], xc, s));
        rc = vmult_internal(h, xc, vc, s);
        if (rc) return rc;
        HIPCHK(h, launch_init_cg(n, rc_, pc, vc, 1, s)); /* r = b - A x0, p = v = 0 */
        double rr = 0.0;
        rc = host_sumsq(h, rc_, nullptr, n, &rr, s);
        if (rc) return rc;
        st[c].bnorm = std::sqrt(bb);
        st[c].eps = tol * st[c].bnorm;
        st[c].r0norm = std::sqrt(rr);
        st[c].flag = st[c].r0norm < st[c].eps ? FLAG_CONV : FLAG_RUN;
        HIPCHK(h, hipMemcpyAsync(h->histM + c * hs, &st[c].r0norm, sizeof(double), hipMemcpyHostToDevice, s));
    }
    HIPCHK(h, hipMemcpyAsync(h->stM, st.data(), sizeof(CGState) * m, hipMemcpyHostToDevice, s));
    IterArgs<double> a{};
    a.L = h->lv;
    a.G = op_geometry(h);
    a.dinv = h->dinv;
    a.r = h->rM;
    a.p = h->pM;
    a.v = h->vM;
    a.x = h->xM;
    a.part = h->partM;
    a.dots = h->dotsM;
    a.st = h->stM;
    a.hist = h->histM;
    a.nshared_blocks = h->nshared_blocks;
    auto running = [&]() {
        for (int c = 0; c < m; ++c)
            if (st[c].flag == FLAG_RUN) return true;
        return false;
    };
    int launched = 0;
    while (running() && launched < maxit) {
        const int chunk = std::min(h->check_every, maxit - launched);
        for (int it = 0; it < chunk; ++it) {
            HIPCHK(h, launch_fused_vec(h->K, MODE_CG | op_flags(h), a, m, n, ps, 8 * nrec, 1, s));
            HIPCHK(h, launch_shared_finish_multi(a, m, n, ps, 8 * nrec, hs, s));
        }
        launched += chunk;
        HIPCHK(h, hipMemcpyAsync(st.data(), h->stM, sizeof(CGState) * m, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
    }
    int first = MFCG_OK;
    for (int c = 0; c < m; ++c) {
        if (zero[c]) {
            HIPCHK(h, hipMemsetAsync(x[c], 0, sizeof(double) * n, s));
        } else {
            HIPCHK(h, launch_reconstruct<double>(n, h->xM + c * n, h->pM + c * n, h->rM + c * n, h->dinv, h->stM + c,
                                                 s));
            HIPCHK(h, launch_int_to_lex<double>(h->lv, h->xM + c * n, x[c], s));
        }
        iters[c] = zero[c] ? 0 : st[c].k;
        status[c] = st[c].flag == FLAG_CONV ? MFCG_OK : (st[c].flag == FLAG_BREAK ? MFCG_EBREAKDOWN : MFCG_ENOTCONV);
        if (first == MFCG_OK && status[c] != MFCG_OK) first = status[c];
    }
    HIPCHK(h, hipStreamSynchronize(s));
    if (true_rel_res) {
        for (int c = 0; c < m; ++c) {
            if (zero[c]) {
                true_rel_res[c] = 0.0;
                continue;
            }
            HIPCHK(h, launch_lex_to_int<double>(h->lv, x[c], h->vin, s));
            int rc = vmult_internal(h, h->vin, h->vout, s);
            if (rc) return rc;
            HIPCHK(h, launch_int_to_lex<double>(h->lv, h->vout, h->vin, s));
            double rr = 0.0;
            rc = host_sumsq(h, b[c], h->vin, n, &rr, s);
            if (rc) return rc;
            true_rel_res[c] = std::sqrt(rr) / st[c].bnorm;
        }
    }
    if (first == MFCG_EBREAKDOWN) return fail(h, first, "breakdown in at least one right-hand side");
    if (first == MFCG_ENOTCONV) return fail(h, first, "maxit reached for at least one right-hand side");
    return MFCG_OK;
}

/* Vector problem (three uncoupled components sharing the operator, the
 * diagonal and the CG scalars): each iteration runs one fused launch over
 * (tile, component) pairs and the shared-node kernel per component, each
 * component writing its own block of inner-product records and shared
 * partial sums, then one finish over all records. */
int mfcg_solve_vector(mfcg_handle h, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                      double *res_hist, double *true_rel_res, void *hip_stream)
{
    if (!h || !b || !x || !iters) return fail(h, MFCG_EINVAL, "null argument");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(h, MFCG_EINVAL, "tol must be finite and >= 0");
    if (maxit < 1) return fail(h, MFCG_EINVAL, "maxit must be >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = h->hl.n;
    const int64_t nrec = h->hl.ntiles + h->nshared_blocks; /* records per component */
    /* the device CG state is reused: a scalar solve in progress ends here */
    h->maxit = 0;
    h->launched = 0;
    if (!h->r3 || !h->p3 || !h->v3 || !h->x3 || !h->dots3 || !h->part3) {
        /* all or nothing: after a failed allocation the next call starts over */
        HIPCHK(h, hipStreamSynchronize(s));
        double *bufs[] = {h->r3, h->p3, h->v3, h->x3, h->dots3, h->part3};
        for (double *q : bufs)
            if (q) HIPCHK(h, hipFree(q));
        h->r3 = h->p3 = h->v3 = h->x3 = h->dots3 = h->part3 = nullptr;
        HIPCHK(h, dalloc(&h->r3, 3 * n));
        HIPCHK(h, dalloc(&h->p3, 3 * n));
        HIPCHK(h, dalloc(&h->v3, 3 * n));
        HIPCHK(h, dalloc(&h->x3, 3 * n));
        HIPCHK(h, dalloc(&h->dots3, 8 * 3 * nrec));
        HIPCHK(h, dalloc(&h->part3, 3 * std::max<int64_t>(1, h->hl.npart)));
        HIPCHK(h, hipMemsetAsync(h->part3, 0, sizeof(double) * 3 * std::max<int64_t>(1, h->hl.npart), s));
    }
    if (maxit > h->hist_cap) {
        HIPCHK(h, hipStreamSynchronize(s));
        HIPCHK(h, hipFree(h->hist));
        h->hist = nullptr;
        h->hist_cap = 0; /* a failed allocation leaves no buffer behind */
        HIPCHK(h, dalloc(&h->hist, (size_t)maxit + 1));
        h->hist_cap = maxit;
    }
    for (int c = 0; c < 3; ++c) HIPCHK(h, launch_lex_to_int<double>(h->lv, b + c * n, h->r3 + c * n, s));
    double bb = 0.0;
    int rc = host_sumsq(h, h->r3, nullptr, 3 * n, &bb, s);
    if (rc) return rc;
    const double bnorm = std::sqrt(bb);
    if (bb == 0.0) {
        HIPCHK(h, hipMemsetAsync(x, 0, sizeof(double) * 3 * n, s));
        HIPCHK(h, hipStreamSynchronize(s));
        *iters = 0;
        if (res_hist) res_hist[0] = 0.0;
        if (true_rel_res) *true_rel_res = 0.0;
        return MFCG_OK;
    }
    /* r = b - A x0, p = v = 0 */
    for (int c = 0; c < 3; ++c) {
        HIPCHK(h, launch_lex_to_int<double>(h->lv, x + c * n, h->x3 + c * n, s));
        rc = vmult_internal(h, h->x3 + c * n, h->v3 + c * n, s);
        if (rc) return rc;
    }
    HIPCHK(h, launch_init_cg(3 * n, h->r3, h->p3, h->v3, 1, s));
    double rr = 0.0;
    rc = host_sumsq(h, h->r3, nullptr, 3 * n, &rr, s);
    if (rc) return rc;
    CGState st{};
    st.eps = tol * bnorm;
    st.bnorm = bnorm;
    st.r0norm = std::sqrt(rr);
    st.maxit = maxit;
    st.flag = st.r0norm < st.eps ? FLAG_CONV : FLAG_RUN;
    HIPCHK(h, hipMemcpyAsync(h->st, &st, sizeof(CGState), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->hist, &st.r0norm, sizeof(double), hipMemcpyHostToDevice, s));
    IterArgs<double> ac[3];
    for (int c = 0; c < 3; ++c) {
        IterArgs<double> &a = ac[c];
        a = IterArgs<double>{};
        a.L = h->lv;
        a.G = op_geometry(h);
        a.dinv = h->dinv;
        a.r = h->r3 + c * n;
        a.p = h->p3 + c * n;
        a.v = h->v3 + c * n;
        a.x = h->x3 + c * n;
        a.part = h->part3 + c * std::max<int64_t>(1, h->hl.npart);
        a.dots = h->dots3 + 8 * c * nrec;
        a.st = h->st;
        a.hist = h->hist;
        a.nshared_blocks = h->nshared_blocks;
    }
    int launched = 0;
    rc = read_state(h, st, s);
    if (rc) return rc;
    while (st.flag == FLAG_RUN && launched < maxit) {
        const int chunk = std::min(h->check_every, maxit - launched);
        for (int it = 0; it < chunk; ++it) {
            /* the three components' tiles in one launch (geometry shared in L2) */
            HIPCHK(h, launch_fused_vec(h->K, MODE_CG | op_flags(h), ac[0], 3, n, std::max<int64_t>(1, h->hl.npart),
                                       8 * nrec, 0, s));
            for (int c = 0; c < 3; ++c) HIPCHK(h, launch_shared_nofinish(ac[c], s));
            HIPCHK(h, launch_finish_parts(ac[0], 3 * nrec, s));
        }
        launched += chunk;
        rc = read_state(h, st, s);
        if (rc) return rc;
    }
    for (int c = 0; c < 3; ++c) {
        HIPCHK(h, launch_reconstruct<double>(n, ac[c].x, ac[c].p, ac[c].r, h->dinv, h->st, s));
        HIPCHK(h, launch_int_to_lex<double>(h->lv, ac[c].x, x + c * n, s));
    }
    if (res_hist) HIPCHK(h, hipMemcpyAsync(res_hist, h->hist, sizeof(double) * (st.k + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    *iters = st.k;
    if (true_rel_res) {
        double tot = 0.0;
        for (int c = 0; c < 3; ++c) {
            HIPCHK(h, launch_lex_to_int<double>(h->lv, x + c * n, h->vin, s));
            rc = vmult_internal(h, h->vin, h->vout, s);
            if (rc) return rc;
            HIPCHK(h, launch_int_to_lex<double>(h->lv, h->vout, h->vin, s));
            double part = 0.0;
            rc = host_sumsq(h, b + c * n, h->vin, n, &part, s);
            if (rc) return rc;
            tot += part;
        }
        *true_rel_res = std::sqrt(tot) / bnorm;
    }
    if (st.flag == FLAG_CONV) return MFCG_OK;
    if (st.flag == FLAG_BREAK) return fail(h, MFCG_EBREAKDOWN, "breakdown: p^T A p <= 0 or non-finite scalar");
    return fail(h, MFCG_ENOTCONV, "maxit reached");
}

int mfcg_solve(mfcg_handle h, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
               double *res_hist, double *true_rel_res, void *hip_stream)
{
    if (!h || !b || !x || !iters) return fail(h, MFCG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = mfcg_cg_begin(h, b, x, tol, maxit, hip_stream);
    if (rc) return rc;
    CGState st{};
    rc = read_state(h, st, s);
    if (rc) return rc;
    while (st.flag == FLAG_RUN && h->launched < maxit) {
        const int chunk = std::min(h->check_every, maxit - h->launched);
        rc = mfcg_cg_iterate(h, chunk, hip_stream);
        if (rc) return rc;
        rc = read_state(h, st, s);
        if (rc) return rc;
    }
    const int status = mfcg_cg_end(h, x, iters, res_hist, hip_stream);
    if (status != MFCG_OK && status != MFCG_ENOTCONV && status != MFCG_EBREAKDOWN) return status;
    if (true_rel_res) {
        if (h->zero_rhs) {
            *true_rel_res = 0.0;
        } else {
            HIPCHK(h, launch_lex_to_int<double>(h->lv, x, h->vin, s));
            rc = vmult_internal(h, h->vin, h->vout, s);
            if (rc) return rc;
            HIPCHK(h, launch_int_to_lex<double>(h->lv, h->vout, h->vin, s));
            double rr = 0.0;
            rc = host_sumsq(h, b, h->vin, h->hl.n, &rr, s);
            if (rc) return rc;
            *true_rel_res = std::sqrt(rr) / h->bnorm;
        }
    }
    return status;
}

/* FP32 copy of the geometry tensor and inverse diagonal plus FP32 work
 * vectors, built on first use. */
static int ensure_fp32(mfcg_ctx *h, hipStream_t s)
{
    if (h->fp32_ready) return MFCG_OK;
    if (h->gll || h->mass || h->q2 || h->qgeom)
        return fail(h, MFCG_EINVAL,
                    "the FP32 operator is built for the Gauss-point Laplacian (k+1 points, stored tensor) only");
    const HostLayout &L = h->hl;
    /* all or nothing: what an earlier failed call left behind is freed first */
    HIPCHK(h, hipStreamSynchronize(s));
    void *olds[] = {h->G32, h->dinv32, h->r32, h->p32, h->v32, h->x32, h->part32, h->dots32, h->st32};
    for (void *q : olds)
        if (q) HIPCHK(h, hipFree(q));
    h->G32 = h->dinv32 = h->r32 = h->p32 = h->v32 = h->x32 = h->part32 = h->dots32 = nullptr;
    h->st32 = nullptr;
    HIPCHK(h, dalloc(&h->G32, L.g_elems));
    HIPCHK(h, dalloc(&h->dinv32, L.n));
    HIPCHK(h, dalloc(&h->r32, L.n));
    HIPCHK(h, dalloc(&h->p32, L.n));
    HIPCHK(h, dalloc(&h->v32, L.n));
    HIPCHK(h, dalloc(&h->x32, L.n));
    HIPCHK(h, dalloc(&h->part32, std::max<int64_t>(1, L.npart)));
    HIPCHK(h, dalloc(&h->dots32, 8 * (L.ntiles + h->nshared_blocks)));
    HIPCHK(h, dalloc(&h->st32, 1));
    HIPCHK(h, hipMemsetAsync(h->part32, 0, sizeof(float) * std::max<int64_t>(1, L.npart), s));
    HIPCHK(h, launch_convert(L.g_elems, h->G, h->G32, s));
    HIPCHK(h, launch_convert(L.n, h->dinv, h->dinv32, s));
    h->fp32_ready = true;
    return MFCG_OK;
}

/* One FP32 segment of the fused CG (Algorithm 5 in single precision:
 * operator, vector updates and inner products) on A d = r32 from d = 0.
 * keep_direction = 0: a fresh CG (p_0 = 0).  keep_direction = 1: the
 * search direction of the previous segment is kept, p_1 = D^{-1} r + beta_in
 * p_prev (the residual was replaced by the FP64 one, the Krylov direction
 * continues).  The segment ends after the first poll at which the
 * recursive residual norm is below inner_tol * rnorm, or after max_inner
 * iterations; d is reconstructed into x32 and the last beta is returned. */
static int fp32_cg(mfcg_ctx *h, double rnorm, double inner_tol, int max_inner, int keep_direction, double beta_in,
                   int *its, double *beta_out, hipStream_t s)
{
    const int64_t n = h->hl.n;
    if (max_inner >= h->hist32_cap) {
        if (h->hist32) HIPCHK(h, hipFree(h->hist32));
        h->hist32 = nullptr;
        h->hist32_cap = 0;
        HIPCHK(h, dalloc(&h->hist32, (size_t)max_inner + 1));
        h->hist32_cap = (int64_t)max_inner + 1;
    }
    HIPCHK(h, hipMemsetAsync(h->x32, 0, sizeof(float) * n, s));
    if (!keep_direction) {
        HIPCHK(h, hipMemsetAsync(h->p32, 0, sizeof(float) * n, s));
        HIPCHK(h, hipMemsetAsync(h->v32, 0, sizeof(float) * n, s));
    }
    CGState st{};
    st.eps = 0.0; /* the host ends the segment; beta is computed in every iteration */
    st.bnorm = rnorm;
    st.r0norm = rnorm;
    st.maxit = max_inner;
    st.beta = keep_direction ? beta_in : 0.0; /* alpha = 0: r stays the replaced residual */
    st.flag = rnorm > 0.0 ? FLAG_RUN : FLAG_CONV;
    HIPCHK(h, hipMemcpyAsync(h->st32, &st, sizeof(CGState), hipMemcpyHostToDevice, s));
    IterArgs<float> a{};
    a.L = h->lv;
    a.G = h->G32;
    a.dinv = h->dinv32;
    a.r = h->r32;
    a.p = h->p32;
    a.v = h->v32;
    a.x = h->x32;
    a.part = h->part32;
    a.dots = h->dots32;
    a.st = h->st32;
    a.hist = h->hist32;
    a.nshared_blocks = h->nshared_blocks;
    int launched = 0;
    double rho = rnorm;
    while (st.flag == FLAG_RUN && launched < max_inner && !(rho < inner_tol * rnorm)) {
        const int chunk = std::min(h->check_every, max_inner - launched);
        for (int it = 0; it < chunk; ++it) {
            HIPCHK(h, launch_fused<float>(h->K, MODE_CG, a, s));
            HIPCHK(h, launch_shared<float>(MODE_CG, a, s));
        }
        launched += chunk;
        HIPCHK(h, hipMemcpyAsync(&st, h->st32, sizeof(CGState), hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        if (st.k > 0) {
            HIPCHK(h, hipMemcpyAsync(&rho, h->hist32 + st.k, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
        }
    }
    HIPCHK(h, launch_reconstruct<float>(n, h->x32, h->p32, h->r32, h->dinv32, h->st32, s));
    *its = st.k;
    if (beta_out) *beta_out = st.beta;
    if (st.flag == FLAG_BREAK) return fail(h, MFCG_EBREAKDOWN, "breakdown in the FP32 inner solve");
    return MFCG_OK;
}

int mfcg_solve_ir(mfcg_handle h, const double *b, double *x, double tol, double inner_tol, int32_t max_outer,
                  int32_t max_inner, int32_t keep_direction, int32_t *outer_its, int32_t *inner_its,
                  double *res_hist, double *true_rel_res, void *hip_stream)
{
    if (!h || !b || !x || !outer_its || !inner_its) return fail(h, MFCG_EINVAL, "null argument");
    if (!(tol > 0.0) || !std::isfinite(tol) || !(inner_tol > 0.0) || !(inner_tol < 1.0))
        return fail(h, MFCG_EINVAL, "need tol > 0 and 0 < inner_tol < 1");
    if (max_outer < 1 || max_inner < 1) return fail(h, MFCG_EINVAL, "max_outer and max_inner must be >= 1");
    if (h->gll || h->mass || h->q2 || h->qgeom)
        return fail(h, MFCG_EINVAL, "mixed precision runs the Gauss-point Laplacian (k+1 points, stored tensor) only");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = ensure_fp32(h, s);
    if (rc) return rc;
    const int64_t n = h->hl.n;
    double *bint = h->vin, *ax = h->vout, *x64 = h->x, *r64 = h->r;
    HIPCHK(h, launch_lex_to_int<double>(h->lv, b, bint, s));
    HIPCHK(h, launch_lex_to_int<double>(h->lv, x, x64, s));
    double bb = 0.0;
    rc = host_sumsq(h, bint, nullptr, n, &bb, s);
    if (rc) return rc;
    const double bnorm = std::sqrt(bb);
    *outer_its = 0;
    *inner_its = 0;
    if (bb == 0.0) {
        HIPCHK(h, hipMemsetAsync(x, 0, sizeof(double) * n, s));
        HIPCHK(h, hipStreamSynchronize(s));
        if (res_hist) res_hist[0] = 0.0;
        if (true_rel_res) *true_rel_res = 0.0;
        return MFCG_OK;
    }
    int status = MFCG_ENOTCONV;
    double prev = 0.0, beta = 0.0;
    int slow = 0;
    for (int outer = 0;; ++outer) {
        /* FP64 residual of the current iterate */
        rc = vmult_internal(h, x64, ax, s);
        if (rc) return rc;
        HIPCHK(h, launch_residual(n, bint, ax, r64, s));
        double rr = 0.0;
        rc = host_sumsq(h, r64, nullptr, n, &rr, s);
        if (rc) return rc;
        const double rn = std::sqrt(rr);
        if (res_hist) res_hist[outer] = rn / bnorm;
        if (true_rel_res) *true_rel_res = rn / bnorm;
        if (rn < tol * bnorm) {
            status = MFCG_OK;
            break;
        }
        if (!std::isfinite(rn)) {
            status = fail(h, MFCG_EBREAKDOWN, "non-finite residual in iterative refinement");
            break;
        }
        if (outer > 0 && rn > 0.1 * prev) {
            if (++slow >= 2) {
                status = fail(h, MFCG_ESTAGNATION, "outer residual stopped decreasing");
                break;
            }
        } else {
            slow = 0;
        }
        if (outer == max_outer) {
            status = fail(h, MFCG_ENOTCONV, "max_outer reached");
            break;
        }
        prev = rn;
        /* inner FP32 solve of A d = r, then x += d in FP64 */
        HIPCHK(h, launch_convert(n, r64, h->r32, s));
        int its = 0;
        /* never reduce further than the outer target needs */
        const double itol = std::min(0.5, std::max(inner_tol, 0.5 * tol * bnorm / rn));
        rc = fp32_cg(h, rn, itol, max_inner, keep_direction && outer > 0 && slow == 0, beta, &its, &beta, s);
        if (rc) return rc;
        *inner_its += its;
        HIPCHK(h, launch_add_correction(n, x64, h->x32, s));
        *outer_its = outer + 1;
    }
    HIPCHK(h, launch_int_to_lex<double>(h->lv, x64, x, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return status;
}

int mfcg_stream_bench(int32_t kind, int64_t n, const double *src, double *dst, int32_t nblocks, void *hip_stream)
{
    if (n < 2 || (n & 1) || !src || !dst || kind < 0 || kind > 15 || ((kind >> 1) & 3) == 3 || nblocks < 1)
        return fail(nullptr, MFCG_EINVAL, "bad stream_bench arguments");
    HIPCHK(nullptr, launch_stream(kind, n, src, dst, nblocks, (hipStream_t)hip_stream));
    return MFCG_OK;
}


/* ------------------------------------------------------------------ */
/* Tile autotuner and batches of independent problems                 */
/* ------------------------------------------------------------------ */

int mfcg_autotune_tile(const mfcg_mesh *mesh, int32_t degree, int32_t iters, int32_t *tile_out, double *ms_out,
                       void *hip_stream)
{
    std::string msg;
    int rc = validate_mesh(mesh, degree, nullptr, msg);
    if (rc) return fail(nullptr, rc, msg);
    if (!tile_out || iters < 1) return fail(nullptr, MFCG_EINVAL, "bad autotune arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    int tx = 0, ty = 0;
    tile_limits(degree, &tx, &ty);
    /* candidates: the compiled maximum extent in x and y; in z 8, 16 or 32
     * cell layers, or the mesh split into 1..12 equal tile layers of at
     * least 2 cells (tile counts that fill the resident workgroup slots
     * evenly; the shallow ones for small meshes); half the x/y extent with
     * 16 layers as a check */
    std::vector<std::array<int, 3>> cand;
    auto add = [&](int hx, int hy, int z) {
        std::array<int, 3> t = {std::min(hx, mesh->cells[0]), std::min(hy, mesh->cells[1]), std::min(z, mesh->cells[2])};
        if (t[2] >= 1 && std::find(cand.begin(), cand.end(), t) == cand.end()) cand.push_back(t);
    };
    for (int z : {8, 16, 32}) add(tx, ty, z);
    for (int m = 1; m <= 12; ++m) {
        const int z = (mesh->cells[2] + m - 1) / m;
        if (z >= 2 && z <= 64) add(tx, ty, z);
    }
    add((tx + 1) / 2, (ty + 1) / 2, 16);
    int64_t n = 1;
    for (int d = 0; d < 3; ++d) n *= (int64_t)mesh->cells[d] * degree + 1;
    double *b = nullptr;
    HIPCHK(nullptr, dalloc(&b, n));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(nullptr, hipEventCreate(&e0));
    HIPCHK(nullptr, hipEventCreate(&e1));
    double best = 1e300;
    std::array<int, 3> bt = cand[0];
    int status = MFCG_OK;
    for (const auto &t : cand) {
        mfcg_options o{};
        o.tile[0] = t[0];
        o.tile[1] = t[1];
        o.tile[2] = t[2];
        mfcg_handle h = nullptr;
        rc = mfcg_setup(mesh, degree, nullptr, &o, hip_stream, &h);
        if (rc) {
            status = rc;
            break;
        }
        float ms = 0.f;
        rc = mfcg_assemble_rhs(h, MFCG_RHS_SINE, nullptr, b, hip_stream);
        if (!rc) rc = mfcg_cg_begin(h, b, nullptr, 0.0, iters + 2, hip_stream);
        if (!rc) rc = mfcg_cg_iterate(h, 2, hip_stream);
        if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = MFCG_EHIP;
        if (!rc) rc = mfcg_cg_iterate(h, iters, hip_stream);
        if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = MFCG_EHIP;
        mfcg_destroy(h);
        if (rc) {
            status = rc;
            break;
        }
        if (ms < best) {
            best = ms;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(b);
    if (status) return fail(nullptr, status, "autotune: a candidate failed");
    for (int d = 0; d < 3; ++d) tile_out[d] = bt[d];
    if (ms_out) *ms_out = best / iters;
    return MFCG_OK;
}

}  // extern "C"

struct mfcg_batch_ctx {
    std::vector<mfcg_ctx *> probs;
    std::vector<std::array<int32_t, 3>> tiles;
    IterArgs<double> *d_args = nullptr;
    int2 *d_items = nullptr;   /* all fused-kernel items, grouped by degree */
    int2 *d_shared = nullptr;  /* shared-node items */
    int *d_active = nullptr;
    CGState *d_states = nullptr; /* gathered solver states of all problems */
    CGState *h_states = nullptr; /* pinned host copy */
    int64_t max_items = 0, max_shared = 0;
    int check_every = 16;
    std::string err;
};

static void batch_release(mfcg_batch_ctx *hb)
{
    for (mfcg_ctx *h : hb->probs)
        if (h) mfcg_destroy(h);
    (void)hipFree(hb->d_args);
    (void)hipFree(hb->d_items);
    (void)hipFree(hb->d_shared);
    (void)hipFree(hb->d_active);
    (void)hipFree(hb->d_states);
    if (hb->h_states) (void)hipHostFree(hb->h_states);
}

static int batch_fail(mfcg_batch_ctx *hb, int code, const std::string &msg)
{
    if (hb) hb->err = msg;
    g_last_error = msg;
    return code;
}

#define BCHK(hb, call)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            (void)hipGetLastError();                                                            \
            return batch_fail((hb), e_ == hipErrorOutOfMemory ? MFCG_ENOMEM : MFCG_EHIP,        \
                              std::string(#call) + ": " + hipGetErrorString(e_));                \
        }                                                                                       \
    } while (0)

static IterArgs<double> iter_args(const mfcg_ctx *h)
{
    IterArgs<double> a{};
    a.L = h->lv;
    a.G = op_geometry(h);
    a.dinv = h->dinv;
    a.r = h->r;
    a.p = h->p;
    a.v = h->v;
    a.x = h->x;
    a.part = h->part;
    a.dots = h->dots;
    a.st = h->st;
    a.hist = h->hist;
    a.nshared_blocks = h->nshared_blocks;
    return a;
}

extern "C" {

}  // extern "C"

/* ------------------------------------------------------------------ */
/* Autotuner cache: one JSON record per tuned case, one record per line */
/* ------------------------------------------------------------------ */

struct TuneKey {
    std::string gpu;
    int k, cells, map;
    std::string prec;
};

static std::string gpu_key()
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string n = std::string(prop.gcnArchName) + "/" + prop.name;
    for (char &c : n)
        if (c == '"' || c == '\\' || (unsigned char)c < 32) c = '_';
    return n;
}

static std::string tune_record(const TuneKey &key, const int tile[3], double ms)
{
    char buf[512];
    snprintf(buf, sizeof(buf),
             "{\"gpu\": \"%s\", \"k\": %d, \"cells\": %d, \"map\": %d, \"precision\": \"%s\", "
             "\"tile\": [%d, %d, %d], \"ms\": %.6g}",
             key.gpu.c_str(), key.k, key.cells, key.map, key.prec.c_str(), tile[0], tile[1], tile[2], ms);
    return buf;
}

/* the record's key part (everything before "tile") identifies the case */
static std::string record_key(const std::string &rec)
{
    const size_t p = rec.find("\"tile\"");
    return p == std::string::npos ? std::string() : rec.substr(rec.find('{'), p - rec.find('{'));
}

static std::vector<std::string> tune_cache_read(const char *path)
{
    std::vector<std::string> recs;
    FILE *f = fopen(path, "r");
    if (!f) return recs;
    char line[1024];
    while (fgets(line, sizeof(line), f)) {
        std::string l(line);
        const size_t a = l.find('{'), b = l.rfind('}');
        if (l.find("\"gpu\"") == std::string::npos || a == std::string::npos || b == std::string::npos) continue;
        recs.push_back(l.substr(a, b - a + 1));
    }
    fclose(f);
    return recs;
}

static bool tune_cache_lookup(const char *path, const TuneKey &key, int tile[3])
{
    const int zero[3] = {0, 0, 0};
    const std::string want = record_key(tune_record(key, zero, 0.0));
    for (const std::string &r : tune_cache_read(path)) {
        if (record_key(r) != want) continue;
        const size_t p = r.find('[', r.find("\"tile\""));
        if (p != std::string::npos && sscanf(r.c_str() + p, "[%d, %d, %d]", &tile[0], &tile[1], &tile[2]) == 3 &&
            tile[0] > 0 && tile[1] > 0 && tile[2] > 0)
            return true;
    }
    return false;
}

/* adds or replaces the case's record; written to a temporary file and
 * renamed, so a reader never sees a partial file */
static void tune_cache_store(const char *path, const TuneKey &key, const int tile[3], double ms)
{
    const std::string rec = tune_record(key, tile, ms), k = record_key(rec);
    std::vector<std::string> recs;
    for (const std::string &r : tune_cache_read(path))
        if (record_key(r) != k) recs.push_back(r);
    recs.push_back(rec);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\"version\": 1, \"entries\": [\n");
    for (size_t i = 0; i < recs.size(); ++i) fprintf(f, "%s%s\n", recs[i].c_str(), i + 1 < recs.size() ? "," : "");
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    if (ok) rename(tmp.c_str(), path);
}

/* autotune: 0 none, 1 per degree; fixed: a tile for every problem (clipped
 * to its mesh) or NULL; cache: autotuner cache path or NULL */
static int batch_setup_impl(int32_t nprob, const mfcg_mesh *meshes, const int32_t *degrees,
                            const double *const *coeffs, int autotune, const int32_t *fixed, const char *cache,
                            void *hip_stream, mfcg_batch *out)
{
    if (!out) return batch_fail(nullptr, MFCG_EINVAL, "null out");
    *out = nullptr;
    if (nprob < 1 || !meshes || !degrees) return batch_fail(nullptr, MFCG_EINVAL, "bad batch arguments");
    for (int i = 0; i < nprob; ++i) {
        std::string msg;
        int rc = validate_mesh(&meshes[i], degrees[i], nullptr, msg);
        if (rc) return batch_fail(nullptr, rc, "problem " + std::to_string(i) + ": " + msg);
    }
    mfcg_batch_ctx *hb = new (std::nothrow) mfcg_batch_ctx();
    if (!hb) return batch_fail(nullptr, MFCG_ENOMEM, "host allocation failed");
    hb->probs.assign(nprob, nullptr);
    hb->tiles.assign(nprob, {0, 0, 0});
    /* one autotuned tile per degree, on a cube of min(largest problem, 48) cells of the first problem's map */
    if (autotune) {
        for (int K = 1; K <= 8; ++K) {
            int first = -1, cmax = 0;
            for (int i = 0; i < nprob; ++i)
                if (degrees[i] == K) {
                    if (first < 0) first = i;
                    cmax = std::max(cmax, std::min(meshes[i].cells[0], std::min(meshes[i].cells[1], meshes[i].cells[2])));
                }
            if (first < 0) continue;
            mfcg_mesh m = meshes[first];
            const int c = std::min(cmax, 48);
            m.cells[0] = m.cells[1] = m.cells[2] = c;
            int32_t t[3];
            const TuneKey key{cache ? gpu_key() : std::string(), K, c, m.map_kind, "fp64"};
            int ct[3], ltx = 0, lty = 0;
            tile_limits(K, &ltx, &lty);
            /* a cached tile beyond this build's compiled x/y extent (a cache
             * written by a build with other tile shapes) counts as a miss */
            if (cache && tune_cache_lookup(cache, key, ct) && ct[0] <= ltx && ct[1] <= lty) {
                for (int d = 0; d < 3; ++d) t[d] = ct[d];
            } else {
                double ms = 0.0;
                int rc = mfcg_autotune_tile(&m, K, 6, t, &ms, hip_stream);
                if (rc) {
                    batch_release(hb);
                    delete hb;
                    return rc;
                }
                if (cache) {
                    const int tt[3] = {t[0], t[1], t[2]};
                    tune_cache_store(cache, key, tt, ms);
                }
            }
            for (int i = 0; i < nprob; ++i)
                if (degrees[i] == K)
                    for (int d = 0; d < 3; ++d) hb->tiles[i][d] = std::min(t[d], meshes[i].cells[d]);
        }
    }
    if (fixed && !autotune)
        for (int i = 0; i < nprob; ++i)
            for (int d = 0; d < 3; ++d) hb->tiles[i][d] = std::min(fixed[d], meshes[i].cells[d]);
    for (int i = 0; i < nprob; ++i) {
        mfcg_options o{};
        for (int d = 0; d < 3; ++d) o.tile[d] = hb->tiles[i][d];
        int rc = mfcg_setup(&meshes[i], degrees[i], coeffs ? coeffs[i] : nullptr, &o, hip_stream, &hb->probs[i]);
        if (rc) {
            std::string m = "problem " + std::to_string(i) + ": " + g_last_error;
            batch_release(hb);
            delete hb;
            return batch_fail(nullptr, rc, m);
        }
        const HostLayout &L = hb->probs[i]->hl;
        for (int d = 0; d < 3; ++d) hb->tiles[i][d] = L.d[d].T;
        hb->max_items += L.ntiles;
        hb->max_shared += hb->probs[i]->nshared_blocks;
    }
    auto bail = [&](hipError_t e) {
        (void)hipGetLastError();
        std::string m = std::string("batch allocation: ") + hipGetErrorString(e);
        batch_release(hb);
        delete hb;
        return batch_fail(nullptr, e == hipErrorOutOfMemory ? MFCG_ENOMEM : MFCG_EHIP, m);
    };
    hipError_t e;
    if ((e = dalloc(&hb->d_args, nprob)) != hipSuccess) return bail(e);
    if ((e = dalloc(&hb->d_items, hb->max_items)) != hipSuccess) return bail(e);
    if ((e = dalloc(&hb->d_shared, hb->max_shared)) != hipSuccess) return bail(e);
    if ((e = dalloc(&hb->d_active, nprob)) != hipSuccess) return bail(e);
    if ((e = dalloc(&hb->d_states, nprob)) != hipSuccess) return bail(e);
    if ((e = hipHostMalloc((void **)&hb->h_states, sizeof(CGState) * nprob, hipHostMallocDefault)) != hipSuccess)
        return bail(e);
    *out = hb;
    return MFCG_OK;
}

extern "C" {

int mfcg_batch_setup(int32_t nprob, const mfcg_mesh *meshes, const int32_t *degrees, const double *const *coeffs,
                     int32_t autotune, void *hip_stream, mfcg_batch *out)
{
    return batch_setup_impl(nprob, meshes, degrees, coeffs, autotune != 0, nullptr, nullptr, hip_stream, out);
}

int mfcg_setup_batch(int32_t nprob, const mfcg_mesh *meshes, const int32_t *degrees, const double *const *coeffs,
                     const mfcg_options *opt, void *hip_stream, mfcg_batch *out)
{
    if (opt && (opt->tile[0] < 0 || opt->tile[1] < 0 || opt->tile[2] < 0))
        return batch_fail(nullptr, MFCG_EINVAL, "tile sizes must be >= 0");
    if (opt && (opt->n_q_1d != 0 || opt->fp32 || opt->quad_rule != MFCG_QUAD_GAUSS || opt->op != MFCG_OP_LAPLACE ||
                opt->geometry != MFCG_GEOM_STORED))
        return batch_fail(nullptr, MFCG_EINVAL, "a batch runs the FP64 Gauss-point Laplacian with the stored tensor");
    const bool fixed = opt && opt->tile[0] > 0 && opt->tile[1] > 0 && opt->tile[2] > 0;
    return batch_setup_impl(nprob, meshes, degrees, coeffs, !fixed, fixed ? opt->tile : nullptr,
                            opt ? opt->tune_cache : nullptr, hip_stream, out);
}

int mfcg_batch_info(mfcg_batch hb, int32_t i, mfcg_handle *h, int32_t *tile)
{
    if (!hb || i < 0 || i >= (int32_t)hb->probs.size()) return batch_fail(hb, MFCG_EINVAL, "bad problem index");
    if (h) *h = hb->probs[i];
    if (tile)
        for (int d = 0; d < 3; ++d) tile[d] = hb->tiles[i][d];
    return MFCG_OK;
}

int mfcg_solve_batch(mfcg_batch hb, const double *const *b, double *const *x, double tol, int32_t maxit,
                     int32_t *iters, int32_t *status, void *hip_stream)
{
    return mfcg_batch_solve(hb, b, x, tol, maxit, iters, status, hip_stream);
}

int mfcg_batch_solve(mfcg_batch hb, const double *const *b, double *const *x, double tol, int32_t maxit,
                     int32_t *iters, int32_t *status, void *hip_stream)
{
    if (!hb || !b || !x || !iters || !status) return batch_fail(hb, MFCG_EINVAL, "null argument");
    const int np = (int)hb->probs.size();
    for (int i = 0; i < np; ++i)
        if (!b[i] || !x[i]) return batch_fail(hb, MFCG_EINVAL, "null vector of problem " + std::to_string(i));
    hipStream_t s = (hipStream_t)hip_stream;
    for (int i = 0; i < np; ++i)
        if (hb->probs[i]->solver != MFCG_SOLVER_FUSED || hb->probs[i]->gll || hb->probs[i]->mass || hb->probs[i]->q2 ||
            hb->probs[i]->qgeom)
            return batch_fail(hb, MFCG_EINVAL,
                              "problem " + std::to_string(i) + ": the batch runs the fused Gauss-quadrature solver only");
    /* every problem starts as mfcg_solve would start it */
    for (int i = 0; i < np; ++i) {
        int rc = mfcg_cg_begin(hb->probs[i], b[i], x[i], tol, maxit, hip_stream);
        if (rc) return batch_fail(hb, rc, "problem " + std::to_string(i) + ": " + hb->probs[i]->err);
    }
    std::vector<IterArgs<double>> args(np);
    for (int i = 0; i < np; ++i) args[i] = iter_args(hb->probs[i]);
    BCHK(hb, hipMemcpyAsync(hb->d_args, args.data(), sizeof(IterArgs<double>) * np, hipMemcpyHostToDevice, s));
    /* the host reads every problem's state with one gather launch and one
     * copy into pinned memory */
    const CGState *st = hb->h_states;
    auto poll = [&]() -> int {
        BCHK(hb, launch_gather_states(hb->d_args, np, hb->d_states, s));
        BCHK(hb, hipMemcpyAsync(hb->h_states, hb->d_states, sizeof(CGState) * np, hipMemcpyDeviceToHost, s));
        BCHK(hb, hipStreamSynchronize(s));
        return MFCG_OK;
    };
    int rc = poll();
    if (rc) return rc;
    std::vector<int2> items, shared;
    std::vector<int> active;
    int launched = 0;
    while (launched < maxit) {
        /* work lists of the problems still running (converged ones drop out) */
        BatchLaunch bl{};
        bl.probs = hb->d_args;
        items.clear();
        shared.clear();
        active.clear();
        int off[10] = {0};
        for (int K = 1; K <= 8; ++K) {
            off[K] = (int)items.size();
            for (int i = 0; i < np; ++i) {
                if (hb->probs[i]->K != K || st[i].flag != FLAG_RUN) continue;
                for (int64_t t = 0; t < hb->probs[i]->hl.ntiles; ++t) items.push_back(make_int2(i, (int)t));
            }
            bl.nitems[K] = (int)items.size() - off[K];
        }
        for (int i = 0; i < np; ++i)
            if (st[i].flag == FLAG_RUN) {
                active.push_back(i);
                for (int q = 0; q < hb->probs[i]->nshared_blocks; ++q) shared.push_back(make_int2(i, q));
            }
        if (active.empty()) break;
        if (!items.empty())
            BCHK(hb, hipMemcpyAsync(hb->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, s));
        if (!shared.empty())
            BCHK(hb, hipMemcpyAsync(hb->d_shared, shared.data(), sizeof(int2) * shared.size(), hipMemcpyHostToDevice, s));
        if (!active.empty())
            BCHK(hb, hipMemcpyAsync(hb->d_active, active.data(), sizeof(int) * active.size(), hipMemcpyHostToDevice, s));
        for (int K = 1; K <= 8; ++K) bl.items[K] = hb->d_items + off[K];
        bl.shared_items = hb->d_shared;
        bl.nshared_items = (int)shared.size();
        bl.active = hb->d_active;
        bl.nactive = (int)active.size();
        const int chunk = std::min(hb->check_every, maxit - launched);
        for (int it = 0; it < chunk; ++it) BCHK(hb, launch_batch_iteration(bl, s));
        launched += chunk;
        rc = poll();
        if (rc) return rc;
    }
    int worst = MFCG_OK;
    for (int i = 0; i < np; ++i) {
        const int r = mfcg_cg_end(hb->probs[i], x[i], &iters[i], nullptr, hip_stream);
        status[i] = r;
        if (r != MFCG_OK && r != MFCG_ENOTCONV && r != MFCG_EBREAKDOWN) return batch_fail(hb, r, hb->probs[i]->err);
        if (r != MFCG_OK && worst == MFCG_OK) worst = r;
    }
    return worst;
}

int mfcg_batch_destroy(mfcg_batch hb)
{
    if (!hb) return MFCG_OK;
    (void)hipDeviceSynchronize();
    batch_release(hb);
    delete hb;
    return MFCG_OK;
}

const char *mfcg_batch_last_error(mfcg_batch hb) { return hb ? hb->err.c_str() : g_last_error.c_str(); }

}  // extern "C"
