/*
 * fused_tile.h -- the fused tile kernel of the Jacobi-PCG iteration
 * (Algorithm 5 of Kronbichler, Sashko, Munch, with the vector updates and
 * inner products embedded in the cell loop of the matrix-free operator,
 * Sec. 5), written for gfx950 (wave64, 160 KB LDS per CU).
 *
 * One iteration k is three launches (this header holds the first; the
 * other two and the launch dispatch are in kernels_cg.hip, the per-degree
 * instantiations in fused_k<K>.hip):
 *
 *  fused_tile_kernel   one workgroup per tile of TX x TY x TZ cells,
 *                      streaming the tile's cell layers along z:
 *     pre   (Alg. 5 "pre" region) on the node planes a layer touches first:
 *           r_k = r_{k-1} - alpha_{k-1} v_{k-1},
 *           p_k = D^{-1} r_k + beta_{k-1} p_{k-1},
 *           x_k = x_{k-2} + alpha_{k-1} p_{k-1}
 *                 + alpha_{k-2}/beta_{k-2} (p_{k-1} - D^{-1} r_{k-1})  (odd k > 1),
 *           written back for tile-interior nodes; recomputed (not written)
 *           for nodes shared with other tiles; p_k staged in an LDS window
 *           of k+1 node planes.  Nodes of the tile's interior entity (one
 *           contiguous run per node plane) take a branch-free path with
 *           uniform base pointers; the other nodes go through the entity
 *           table.
 *     cell  Eq. 5 by sum factorisation: gather from the window, 1D
 *           interpolations to the Gauss points and collocation derivatives
 *           (Sec. 2, sum factorisation), G_q = a w det J J^{-1} J^{-T}
 *           applied per quadrature point, transposed contractions.  Each
 *           thread owns one 1D line of a cell per pass; lines of other
 *           directions are exchanged through LDS.
 *     sum   v = sum of the cell contributions (Eq. 4), in a fixed order.
 *     post  (Alg. 5 "post" region) after the last contribution to a node
 *           (Sec. 5.1): the seven partial sums gamma, a, b, c, d, e, f for
 *           tile-interior nodes, v written once; nodes shared with other
 *           tiles get this tile's partial sum in `part`.
 *
 *  shared_node_kernel  grid-stride over shared and Dirichlet nodes: adds the
 *                      partial sums in a fixed slot order, applies pre and
 *                      post there, writes per-block partial inner products.
 *  finish_kernel       one block: reduces all per-block partials in a fixed
 *                      order and computes alpha_k, beta_k and the convergence
 *                      test on the device (no host round trip).
 *
 * Every reduction and every summation of partial contributions runs in a
 * fixed order, so a solve is bitwise reproducible.
 */
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cg_common.h"
#include "kernels.h"
#include "tables_ct.h"

namespace mfcg {

/* ------------------------------------------------------------------ */
/* Per-degree configuration (compile time)                             */
/* ------------------------------------------------------------------ */

/* TX, TY: compiled maximum tile extent in x and y (cells); WG: workgroup
 * size; GPREF: where a layer's geometry tensor is loaded (0: in the pass
 * that applies it, 1: before the x and z derivative passes, held in
 * registers across them); OCC: workgroups per CU the register allocator
 * aims for; CARRY: r_k and D^{-1} of a node kept in registers from its pre
 * to its post (1) or re-read there (0).  Chosen per degree by timing on
 * MI355X (k = 5: 4x3-cell tiles on 448 threads, 432 lines per pass, were
 * 16% faster per iteration than 3x3 tiles on 384 threads, 324 lines; k = 3:
 * 8x4 tiles on 512 threads, every thread busy, 3-8% faster than 5x5 tiles
 * at three workgroups per CU, 21% with the quadratic geometry, 10% slower
 * with k+2 points; k = 8: 2x1 tiles on 192 threads, four workgroups per CU,
 * 31% faster than 2x2 tiles on 384 threads at two per CU). */
template <int K>
struct Cfg;
template <> struct Cfg<1> { static constexpr int TX = 8, TY = 8, WG = 256, GPREF = 0, OCC = 2, CARRY = 0; };
template <> struct Cfg<2> { static constexpr int TX = 8, TY = 8, WG = 576, GPREF = 0, OCC = 2, CARRY = 0; };
template <> struct Cfg<3> { static constexpr int TX = 8, TY = 4, WG = 512, GPREF = 0, OCC = 2, CARRY = 1; };
template <> struct Cfg<4> { static constexpr int TX = 4, TY = 4, WG = 448, GPREF = 0, OCC = 2, CARRY = 1; };
template <> struct Cfg<5> { static constexpr int TX = 4, TY = 3, WG = 448, GPREF = 0, OCC = 2, CARRY = 1; };
template <> struct Cfg<6> { static constexpr int TX = 2, TY = 2, WG = 256, GPREF = 0, OCC = 2, CARRY = 1; };
template <> struct Cfg<7> { static constexpr int TX = 2, TY = 2, WG = 256, GPREF = 1, OCC = 2, CARRY = 1; };
template <> struct Cfg<8> { static constexpr int TX = 2, TY = 1, WG = 192, GPREF = 0, OCC = 4, CARRY = 0; };

inline void tile_limits_impl(int K, int *tx, int *ty)
{
    static const int x[9] = {0, 8, 8, 8, 4, 4, 2, 2, 2}, y[9] = {0, 8, 8, 4, 4, 3, 2, 2, 1};
    const bool ok = K >= 1 && K <= 8;
    *tx = ok ? x[K] : 0;
    *ty = ok ? y[K] : 0;
}

inline int fused_block_size_impl(int K)
{
    static const int w[9] = {0, 256, 576, 512, 448, 448, 256, 256, 192};
    return (K >= 1 && K <= 8) ? w[K] : 0;
}

/* minimum waves per SIMD requested from the register allocator */
/* build-time overrides of the per-degree choices (timing experiments) */
#ifdef MFCG_OCC
#define MFCG_OCC_OF(K) (MFCG_OCC)
#else
#define MFCG_OCC_OF(K) (Cfg<K>::OCC)
#endif
/* geometry loads issued before the derivative passes (1) or in the G pass (0) */
#ifdef MFCG_GPREF
#define MFCG_GPREF_OF(K) (MFCG_GPREF)
#else
#define MFCG_GPREF_OF(K) (Cfg<K>::GPREF)
#endif
#define MFCG_WPE_MIN(K) ((MFCG_OCC_OF(K) * Cfg<K>::WG / 64 + 3) / 4)
/* r_k and D^{-1} kept in registers from a node's pre to its post */
#ifdef MFCG_CARRY
#define MFCG_CARRY_OF(K) (MFCG_CARRY)
#else
#define MFCG_CARRY_OF(K) (Cfg<K>::CARRY)
#endif
/* the k+2-point variants: no more waves than their larger cell scratch
 * lets fit per CU (LDS per workgroup 32 KB at k = 1, 83 KB at k = 2, 86 KB
 * at k = 3 and 94 KB at k = 5, one workgroup per CU, 77 KB at k = 4, 49 KB
 * at k = 6, 69 KB at k = 7), geometry loads in the G pass */
constexpr int WPE_Q2[8] = {0, 2, 3, 2, 4, 2, 2, 2};
/* the quadratic-geometry variants hold the cell's contracted geometry (27
 * values per line) through the G pass: they ask for as many waves as their
 * register use allows without heavy spills (k = 3: 3 waves per SIMD was 4%
 * faster than 4, k = 4: 4 was 3% faster than 3), at k = 2 as their LDS
 * allows */
constexpr int WPE_QG[9] = {0, 2, 3, 3, 4, 2, 2, 2, 2};
/* the mass operator with quadratic geometry (no derivative passes) */
constexpr int WPE_QGM[9] = {0, 2, 3, 4, 4, 3, 2, 2, 2};
/* both: the k+2 cell buffers plus the staged geometry fit one workgroup per
 * CU at k = 3, 4 and 5 */
constexpr int WPE_QGQ2[8] = {0, 2, 3, 2, 2, 2, 2, 2};
#define MFCG_WPE_MIN_Q(K, QX, OPV)                                                                                   \
    ((QX) ? (((OPV) == OPV_LAPLACE_QGEOM || (OPV) == OPV_MASS_QGEOM) ? WPE_QGQ2[(K) < 8 ? (K) : 0]                   \
                                                                      : WPE_Q2[(K) < 8 ? (K) : 0])                   \
          : ((OPV) == OPV_LAPLACE_QGEOM ? WPE_QG[(K) < 9 ? (K) : 0]                                                 \
                                        : ((OPV) == OPV_MASS_QGEOM ? WPE_QGM[(K) < 9 ? (K) : 0] : MFCG_WPE_MIN(K))))
/* the batch kernel reads its arguments through the global-address-space
 * view and needs the registers of the single-problem kernel */
#define MFCG_WPE_MIN_BATCH(K) MFCG_WPE_MIN(K)

/* ------------------------------------------------------------------ */
/* Helpers                                                             */
/* ------------------------------------------------------------------ */

/* Workgroups are dispatched round-robin over the 8 XCDs (separate L2s).
 * Map consecutive blocks of one XCD to consecutive tiles so that tiles
 * sharing faces mostly run under the same L2. */
__device__ inline int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t X = 8;
    const int64_t q = nb / X, r = nb % X;
    const int64_t x = b % X, i = b / X;
    return x * q + (x < r ? x : r) + i;
}

/* The batch's per-problem arguments live in device memory that no kernel
 * writes during a launch: read them through the constant address space
 * (scalar loads). */
template <typename A>
__device__ __forceinline__ const A *const_view(const A *p)
{
    return (const A *)(const __attribute__((address_space(4))) A *)p;
}

/* Division by a divisor fixed for a workgroup, for dividends below 2^16:
 * q = floor(n * ceil(2^32 / d) / 2^32) is exact when n, d < 2^16. */
struct FastDiv {
    uint32_t d, m;
    __device__ __forceinline__ explicit FastDiv(uint32_t dd)
        : d(dd), m(dd > 1 ? (uint32_t)((0x100000000ull + dd - 1) / dd) : 0u) {}
    __device__ __forceinline__ int div(int n) const { return d > 1 ? (int)__umulhi((uint32_t)n, m) : n; }
    __device__ __forceinline__ int mod(int n) const { return n - div(n) * (int)d; }
};

/* A value known to be equal in all lanes, moved to scalar registers. */
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

/* The geometry tensor is streamed once per iteration: its loads carry the
 * non-temporal hint so that they do not displace the vector lines that are
 * reused within the iteration (measured: 1.5-2% off the fused kernel at
 * Q4, 64^3, and 0.045 GB less HBM traffic per launch).  The vector kernel,
 * whose three components read each tensor line in turn, keeps plain loads
 * so that L2 holds the lines for the second and third reads. */
template <bool NT, typename T>
__device__ __forceinline__ T gload(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

/* t = sum_j M(q, j) u[j] (row q of a 1D table M given by coef) and
 * t = sum_q M(q, m) w[q] (column m), unrolled with the table entries as
 * compile-time constants: exactly-zero entries are skipped and unit
 * entries added, which changes no result (with k + 1 Gauss points and even
 * k, the centre Gauss point is the centre GLL node, so one row of the
 * interpolation matrix is a unit row, and the centre entry of the
 * collocation derivative is zero). */
template <typename T, int N, typename F>
__device__ __forceinline__ T row_dot(F coef, int q, const T (&u)[N])
{
    T t = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const T c = coef(q, j);
        if (c == (T)1)
            t += u[j];
        else if (c != (T)0)
            t = fma(c, u[j], t);
    }
    return t;
}

template <typename T, int N, typename F>
__device__ __forceinline__ T col_dot(F coef, int m, const T (&w)[N])
{
    T t = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const T c = coef(q, m);
        if (c == (T)1)
            t += w[q];
        else if (c != (T)0)
            t = fma(c, w[q], t);
    }
    return t;
}

/* ------------------------------------------------------------------ */
/* Fused tile kernel                                                   */
/* ------------------------------------------------------------------ */

/* Operator variants of the fused kernel: the Laplacian on the Gauss points
 * (default), the Laplacian with quadrature on the GLL nodes (collocation:
 * the interpolation passes are the identity and are skipped), the mass
 * operator on the Gauss points (no derivative passes; component 0 of the
 * stored tensor holds a_e w_q det J_q), and the Laplacian with quadratic
 * geometry (Sec. 2.2): the tensor a_e w_q det J_q J_q^{-1} J_q^{-T} is
 * computed at each Gauss point from the cell's 27 interpolation points
 * instead of being loaded; likewise a_e w_q det J_q for the mass operator
 * with quadratic geometry. */
enum OpVariant : int { OPV_LAPLACE = 0, OPV_LAPLACE_GLL = 1, OPV_MASS = 2, OPV_LAPLACE_QGEOM = 3, OPV_MASS_QGEOM = 4 };

/* One tile of one problem: the pre / cell / sum / post passes over the
 * tile's cell layers (called by one whole workgroup).  QX = 1: k + 2
 * Gauss points per direction instead of k + 1 (Gauss variants only); the
 * passes on the quadrature grid then run over (k + 2)^2 lines per cell and
 * the interpolation passes map k + 1 values to k + 2 and back. */
template <int K, typename T, int MODE, int OPV = OPV_LAPLACE, bool NTG = true, int QX = 0, typename ARGS>
__device__ __forceinline__ void fused_tile(const ARGS &a, const int64_t tile)
{
    constexpr bool GLLQ = OPV == OPV_LAPLACE_GLL, MASS = OPV == OPV_MASS || OPV == OPV_MASS_QGEOM,
                   QGEOM = OPV == OPV_LAPLACE_QGEOM || OPV == OPV_MASS_QGEOM;
    static_assert(QX == 0 || (QX == 1 && !GLLQ && K <= 7), "k+2 points: Gauss rules up to k = 7");
    constexpr int NG = MASS ? 1 : 6; /* tensor components read */
    /* when the geometry loads are issued: 0 in the G pass, 1 before the
     * derivative passes, 2 before the pre pass (measured on MI355X with the
     * present kernel at k = 4: holding a whole layer's tensor in registers,
     * whether issued one layer ahead or all at once in the G pass, costs
     * more in occupancy than it saves in latency: 0.60-0.77 ms against
     * 0.584 ms per launch) */
    constexpr int GPF = (QX || QGEOM) ? 0 : MFCG_GPREF_OF(K);
    constexpr int n = K + 1, n2 = n * n;
    /* nq points per direction; the cell scratch holds nq^3 values with the
     * strides (1, nq, nq^2) in every stage (fewer entries used where a
     * direction still has n values) */
    constexpr int nq = n + QX, q2 = nq * nq, CS = nq * nq * nq, nnq = n * nq;
    constexpr int WG = Cfg<K>::WG;
    constexpr int NLC = Cfg<K>::TX * Cfg<K>::TY;
    constexpr int RA = (NLC * n2 + WG - 1) / WG;  /* lines of the F1 and B7 passes */
    constexpr int RB = (NLC * nnq + WG - 1) / WG; /* F2 and B6 */
    constexpr int R = (NLC * q2 + WG - 1) / WG;   /* passes on the quadrature grid */
    constexpr int PNM = (Cfg<K>::TX * K + 1) * (Cfg<K>::TY * K + 1);
    constexpr int NS = (K * PNM + WG - 1) / WG;
    constexpr int NC = (PNM + WG - 1) / WG;
    /* compile-time 1D tables: S (GLL basis at Gauss points, nq x n), D
     * (collocation derivative on the Gauss points, nq x nq) */
    constexpr ct::Tab<n> TT = ct::make_tab<n, GLLQ>();
    constexpr ct::Tab2<n, nq> TQ = QX ? ct::make_tab2<n, nq>() : ct::Tab2<n, nq>{};
    constexpr auto cS = [](int q, int i) { return QX ? (T)TQ.S[q * n + i] : (T)TT.S[q * n + i]; };
    constexpr auto cD = [](int q, int m) { return QX ? (T)TQ.D[q * nq + m] : (T)TT.D[q * n + m]; };
    /* Gauss points and weights on [0,1] */
    constexpr auto cxq = [](int q) { return QX ? (T)TQ.xq[q] : (T)TT.xq[q]; };
    constexpr auto cwq = [](int q) { return QX ? (T)TQ.wq[q] : (T)TT.wq[q]; };

    __shared__ T win[(K + 1) * PNM];
    __shared__ T TA[NLC * CS];
    /* cell scratch; TB[NLC * CS] stays 0: the sum over the cells around a
     * node reads it for the cells that do not exist */
    __shared__ T TB[NLC * CS + 1];
    __shared__ T cv[2 * PNM];
    /* quadratic geometry of the current layer's cells */
    __shared__ T XS[QGEOM ? NLC * QGEOM_STRIDE : 1];
    /* quadratic geometry, CG modes at k = 4: the inner products flushed per
     * layer, one slot per wave, so that the accumulators are not held through
     * the geometry evaluation (0.79 instead of 0.90 ms per iteration; at the
     * other degrees, which do not spill, the flush costs more than it saves) */
    constexpr bool FLUSH = OPV == OPV_LAPLACE_QGEOM && mode_is_cg(MODE) && K == 4;
    __shared__ T wacc[FLUSH ? 8 * (WG / 64) : 1];
    __shared__ T red[8 * (WG / 64)];
    __shared__ EntityRef ent[27];
    /* per node of the tile's xy plane: x = entity class in x,y (dx + 3 dy)
     * | stride of the entity's z index << 8, y = offset of (x,y) inside the
     * entity, z/w = offsets into the cell scratch of the (up to) 4 cells
     * around the node (16 bits each, 0xffff: no such cell), cell order
     * (-x,-y), (+x,-y), (-x,+y), (+x,+y) */
    __shared__ int4 desc[PNM];
    /* the nodes of a tile node plane that lie on the tile's side faces (the
     * "ring": every node of the plane outside the interior entity), in the
     * order bottom row, top row, left column, right column */
    constexpr int RINGM = 2 * (Cfg<K>::TX + Cfg<K>::TY) * K;
    __shared__ int16_t ring[RINGM];

    const int tid0 = threadIdx.x;
    const TileDesc td = a.L.tiles[tile];
    if (tid0 < 27) ent[tid0] = a.L.tile_ent[tile * 27 + tid0];
    /* The thread index is re-made opaque to the compiler at every phase of
     * the layer loop: all per-thread index arithmetic is then recomputed
     * where it is used instead of being hoisted out of the loop and held in
     * registers across all layers (which doubles the register footprint
     * and halves the number of resident workgroups). */
    int tid = tid0;

    T alpha = 0, beta = 0, ratio = 0;
    bool xupd = false;
    if (mode_is_cg(MODE)) {
        alpha = (T)a.st->alpha;
        beta = (T)a.st->beta;
        ratio = (T)a.st->ratio;
        const int kk = a.st->k + 1;
        xupd = (kk > 1) && (kk & 1);
    }

    const int TXa = td.nc[0], TYa = td.nc[1], TZa = td.nc[2];
    const int EX = TXa * K, EY = TYa * K, EZ = TZa * K;
    const int PW = EX + 1;
    const int PN = (EX + 1) * (EY + 1);
    const int nlines = TXa * TYa * q2;
    const int nlA = QX ? TXa * TYa * n2 : nlines, nlB = QX ? TXa * TYa * nnq : nlines;
    const int gcomp = CS * TXa * TYa; /* stride between components of G in a layer */
    const int gq = TXa * TYa * q2;    /* stride of the y-index of G in a component */
    const FastDiv dPW(PW), dPN(PN), dTX(TXa);
    for (int node = tid0; node < PN; node += WG) {
        const int by = dPW.div(node), ax = node - by * PW;
        const int dx = ax == 0 ? 0 : (ax == EX ? 2 : 1);
        const int dy = by == 0 ? 0 : (by == EY ? 2 : 1);
        const int sx = dx == 1 ? EX - 1 : 1, sy = dy == 1 ? EY - 1 : 1;
        const int lx = dx == 1 ? ax - 1 : 0, ly = dy == 1 ? by - 1 : 0;
        const int cx1 = ax / K, cy1 = by / K;
        const bool xl = (ax % K) == 0 && cx1 > 0, xr = cx1 < TXa;
        const bool yl = (by % K) == 0 && cy1 > 0, yr = cy1 < TYa;
        auto off = [&](int cx, int cy) { return (cx + TXa * cy) * CS + (ax - cx * K) + nq * (by - cy * K); };
        const int o00 = (xl && yl) ? off(cx1 - 1, cy1 - 1) : 0xffff;
        const int o01 = (xr && yl) ? off(cx1, cy1 - 1) : 0xffff;
        const int o10 = (xl && yr) ? off(cx1 - 1, cy1) : 0xffff;
        const int o11 = (xr && yr) ? off(cx1, cy1) : 0xffff;
        desc[node] = make_int4((dx + 3 * dy) | ((sx * sy) << 8), lx + sx * ly, o00 | (o01 << 16), o10 | (o11 << 16));
    }
    /* LDS offsets of the lines this thread owns in every pass (k + 1 points
     * per direction: all passes split a layer's cells into the same
     * (cell, 2D index) lines): z-lines oZ = c CS + rem, x-lines oX =
     * c CS + nq rem, y-lines oY = c CS + i + nq^2 z, and the window position
     * oW of the line's node column for the gather; computed once per tile
     * instead of in every pass */
    int oZ[R], oX[R], oY[R], oW[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int l = tid0 + WG * rr;
        const int c = l / q2, rem = l - c * q2, i = rem % nq, z = rem / nq;
        const int cy = dTX.div(c), cx = c - cy * TXa;
        oZ[rr] = c * CS + rem;
        oX[rr] = c * CS + nq * rem;
        oY[rr] = c * CS + i + q2 * z;
        oW[rr] = cx * K + i + PW * (cy * K + z);
    }
    for (int r = tid0; r < 2 * (EX + EY); r += WG) {
        int node;
        if (r <= EX)
            node = r;
        else if (r < 2 * (EX + 1))
            node = (r - (EX + 1)) + PW * EY;
        else if (r < 2 * (EX + 1) + EY - 1)
            node = PW * (1 + r - 2 * (EX + 1));
        else
            node = EX + PW * (2 + r - 2 * (EX + 1) - EY);
        ring[r] = (int16_t)node;
    }
    if (tid0 == 0) TB[NLC * CS] = 0;
    if (FLUSH && tid0 < 8 * (WG / 64)) wacc[tid0] = 0;
    __syncthreads();

    /* Tile-interior nodes (the interior entity, always of kind I) take a
     * branch-free path: its nodes of interior node planes zz = 1..EZ-1 are
     * one contiguous run per plane, (EX-1)(EY-1) nodes, x fastest, so the
     * f-th interior node from plane zz0 on lies at vector index
     * vbase + (zz0 - 1) SXY + f; the other nodes of a plane (the ring) and the
     * tile's bottom and top planes take the general path through the entity
     * table.  Base pointers are uniform (scalar registers) and offsets 32-bit. */
    const int SXI = EX - 1, SXY = SXI * (EY - 1), NRING = 2 * (EX + EY);
    const int64_t vb13 = uniform64(ent[13].vbase);
    const bool fast = __builtin_amdgcn_readfirstlane(ent[13].kind) == KIND_I && SXY > 0;
    const FastDiv dSXY(SXY > 0 ? SXY : 1), dSXI(SXI > 0 ? SXI : 1), dRING(NRING);
    /* window position of interior node rem of a plane: (lx + 1) + PW (ly + 1) */
    auto inode = [&](int rem) {
        const int ly = dSXI.div(rem);
        return rem + 2 * ly + PW + 1;
    };

    T acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = 0;

    /* element offset, kind and partial-sum offset of the node with xy
     * descriptor dsc on tile plane zz; vectors and partial arrays hold fewer
     * than 2^31 entries */
    auto locate = [&](const int4 &dsc, int zz, int &idx, int &kind, int &pidx) {
        const int dz = zz == 0 ? 0 : (zz == EZ ? 2 : 1);
        const int lz = dz == 1 ? zz - 1 : 0;
        const EntityRef &e = ent[(dsc.x & 0xff) + 9 * dz];
        const int loc = dsc.y + (dsc.x >> 8) * lz;
        idx = (int)e.vbase + loc;
        kind = e.kind;
        pidx = (int)e.pbase + loc;
    };

    /* Algorithm 5's pre, split in two so that a thread issues the loads of
     * all its nodes of a pass before it waits for any of them (one memory
     * round trip per pass instead of one per node): pre_load reads the old
     * r, v, p, D^{-1} (and x on the iterations that update it), pre_apply
     * computes r_k and p_k, writes them back for tile-interior nodes (shared
     * nodes are only recomputed) and returns p_k (0 on Dirichlet nodes);
     * r_k and D^{-1} go to rk, dk (kept in registers for the node's post) */
    struct PreIn {
        T r0, v0, p0, dv, x0;
        int idx, kind;
    };
    auto pre_load = [&](int node, int zz, PreIn &in) {
        int pidx;
        locate(desc[node], zz, in.idx, in.kind, pidx);
        in.r0 = in.v0 = in.p0 = in.x0 = 0;
        in.dv = 1;
        if (in.kind == KIND_C) return;
        if (MODE == MODE_VMULT) {
            in.p0 = a.src[in.idx];
            return;
        }
        in.r0 = a.r[in.idx];
        in.v0 = a.v[in.idx];
        in.p0 = a.p[in.idx];
        if (MODE != MODE_CG_NOPREC) in.dv = a.dinv[in.idx];
        if (xupd && in.kind == KIND_I) in.x0 = a.x[in.idx];
    };
    auto pre_apply = [&](const PreIn &in, T &rk, T &dk) -> T {
        if (in.kind == KIND_C) return (T)0;
        if (MODE == MODE_VMULT) return in.p0;
        T rn, pn;
        pre_update(in.r0, in.v0, in.p0, in.dv, alpha, beta, rn, pn);
        rk = rn;
        dk = in.dv;
        if (in.kind == KIND_I) {
            a.r[in.idx] = rn;
            a.p[in.idx] = pn;
            if (xupd) a.x[in.idx] = x_update(in.x0, in.r0, in.p0, in.dv, alpha, ratio);
        }
        return pn;
    };

    /* v of a layer node summed over the cells around it, fixed order */
    auto sum_cells = [&](const int4 &dsc, int zl) -> T {
        const int o00 = dsc.z & 0xffff, o01 = (int)((unsigned)dsc.z >> 16);
        const int o10 = dsc.w & 0xffff, o11 = (int)((unsigned)dsc.w >> 16);
        const int zo = q2 * zl;
        const T v00 = TB[o00 != 0xffff ? o00 + zo : NLC * CS];
        const T v01 = TB[o01 != 0xffff ? o01 + zo : NLC * CS];
        const T v10 = TB[o10 != 0xffff ? o10 + zo : NLC * CS];
        const T v11 = TB[o11 != 0xffff ? o11 + zo : NLC * CS];
        return ((v00 + v01) + v10) + v11;
    };

    /* post on one node: r_k and D^{-1} from the registers of this thread's
     * pre of the node (reg = true) or re-read (the tile's layer-top plane,
     * whose pre ran in the layer below under another thread mapping), p_k
     * from the window */
    auto post_node = [&](const int4 &dsc, int node, int zz, int slot, T v, bool reg, T rk, T dk) {
        int idx, kind, pidx;
        locate(dsc, zz, idx, kind, pidx);
        if (kind == KIND_S) {
            a.part[pidx] = v;
        } else if (kind == KIND_I) {
            if (MODE == MODE_VMULT) {
                a.dst[idx] = v;
            } else {
                /* the quadratic-geometry G pass needs the registers at k <= 4
                 * (k = 4: 0.90 instead of 1.01 ms per iteration): re-read */
                const bool use = MFCG_CARRY_OF(K) && !(OPV == OPV_LAPLACE_QGEOM && K <= 4) && reg;
                const T rn = use ? rk : a.r[idx];
                const T dv = MODE == MODE_CG_NOPREC ? (T)1 : (use ? dk : a.dinv[idx]);
                const T pn = win[slot * PNM + node];
                const T zr = dv * rn, zv = dv * v;
                acc[0] += rn * rn;
                acc[1] += pn * v;
                acc[2] += rn * v;
                acc[3] += v * v;
                acc[4] += rn * zr;
                acc[5] += rn * zv;
                acc[6] += v * zv;
                a.v[idx] = v;
            }
        }
    };

    /* fast-path nodes per thread: of a layer's interior planes (pre and
     * post) and of one interior plane (the post of a layer's bottom plane) */
    constexpr int SXYM = (Cfg<K>::TX * K - 1) * (Cfg<K>::TY * K - 1);
    constexpr int NFI = (K * SXYM + WG - 1) / WG;
    constexpr int NF0 = (SXYM + WG - 1) / WG;
    /* r_k and D^{-1} of the fast-path nodes this thread pre-processes, held
     * until their post (except where the G pass needs the registers) */
    constexpr bool CARRYF = MFCG_CARRY_OF(K) && !(OPV == OPV_LAPLACE_QGEOM && K <= 4);
    T kr[NFI], kd[NFI];
#pragma unroll
    for (int s = 0; s < NFI; ++s) kr[s] = kd[s] = 0;
    T rdummy, ddummy;

    /* bottom plane of the tile into the window (general path) */
    {
        PreIn in[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int node = tid + WG * c;
            in[c].kind = KIND_C;
            if (node < PN) pre_load(node, 0, in[c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int node = tid + WG * c;
            if (node < PN) win[node] = pre_apply(in[c], rdummy, ddummy);
        }
    }

    T gp[R][6][nq];
#pragma unroll 1
    for (int L = 0; L < TZa; ++L) {
        const int s0 = (L * K) % (K + 1);
        asm volatile("" : "+v"(tid)); /* see above */
        const T *Gl = a.G + td.gbase + (int64_t)L * 6 * gcomp;
        if (QGEOM) {
            /* this layer's cells: the previous layer's last reads of XS
             * were followed by barriers */
            const T *Xl = a.G + td.gbase / (6 * CS) * QGEOM_STRIDE + (int64_t)L * TXa * TYa * QGEOM_STRIDE;
            for (int e = tid; e < TXa * TYa * QGEOM_STRIDE; e += WG) XS[e] = Xl[e];
        }
        if (GPF == 2) {
            /* G of this layer issued first: its latency overlaps the pre loads */
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int l = tid + WG * rr;
#pragma unroll
                for (int j = 0; j < nq; ++j)
#pragma unroll
                    for (int c = 0; c < NG; ++c) gp[rr][c][j] = (l < nlines) ? gload<NTG>(&Gl[c * gcomp + j * gq + l]) : (T)0;
            }
        }
        /* ---- pre on the planes this layer touches first ---- */
        /* interior planes among L K + 1 .. L K + K (K - 1 in the last layer) */
        const int nzi = min(K, EZ - 1 - L * K);
        const int nf = fast ? nzi * SXY : 0;
        /* vector index of the first interior node of plane L K + 1 */
        const int64_t fb = vb13 + (int64_t)(L * K) * SXY;
        /* general-path nodes of the layer: the rings of the interior planes,
         * then whole planes (the tile's top plane) */
        const int NR = fast ? nzi * NRING + (K - nzi) * PN : K * PN;
        auto gdecode = [&](int f, int &zl, int &node) {
            if (fast && f < nzi * NRING) {
                const int zq = dRING.div(f);
                zl = 1 + zq;
                node = ring[f - zq * NRING];
            } else {
                const int f2 = f - (fast ? nzi * NRING : 0);
                const int zq = dPN.div(f2);
                zl = 1 + (fast ? nzi : 0) + zq;
                node = f2 - zq * PN;
            }
        };
        {
            /* fast path: all loads of the thread's nodes, then the updates */
            T r0[NFI], v0[NFI], p0[NFI], d0[NFI], x0[NFI];
            const uint32_t ob = (uint32_t)sizeof(T);
            auto at = [&](const T *base, int f) -> const T & {
                return *(const T *)((const char *)(base + fb) + (uint32_t)f * ob);
            };
            auto atw = [&](T *base, int f) -> T & { return *(T *)((char *)(base + fb) + (uint32_t)f * ob); };
#pragma unroll
            for (int s = 0; s < NFI; ++s) {
                const int f = tid + WG * s;
                r0[s] = v0[s] = p0[s] = x0[s] = 0;
                d0[s] = 1;
                if (f < nf) {
                    if (MODE == MODE_VMULT) {
                        p0[s] = at(a.src, f);
                    } else {
                        r0[s] = at(a.r, f);
                        v0[s] = at(a.v, f);
                        p0[s] = at(a.p, f);
                        if (MODE != MODE_CG_NOPREC) d0[s] = at(a.dinv, f);
                        if (xupd) x0[s] = at(a.x, f);
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < NFI; ++s) {
                const int f = tid + WG * s;
                if (f < nf) {
                    T pn = p0[s];
                    if (MODE != MODE_VMULT) {
                        T rn;
                        pre_update(r0[s], v0[s], p0[s], d0[s], alpha, beta, rn, pn);
                        kr[s] = rn;
                        kd[s] = d0[s];
                        atw(a.r, f) = rn;
                        atw(a.p, f) = pn;
                        if (xupd) atw(a.x, f) = x_update(x0[s], r0[s], p0[s], d0[s], alpha, ratio);
                    }
                    const int zq = dSXY.div(f);
                    int slot = s0 + 1 + zq;
                    if (slot > K) slot -= K + 1;
                    win[slot * PNM + inode(f - zq * SXY)] = pn;
                }
            }
        }
        {
            /* general path (one node at a time) */
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int f = tid + WG * s;
                if (f < NR) {
                    int zl, node;
                    gdecode(f, zl, node);
                    PreIn in;
                    pre_load(node, L * K + zl, in);
                    int slot = s0 + zl;
                    if (slot > K) slot -= K + 1;
                    win[slot * PNM + node] = pre_apply(in, rdummy, ddummy);
                }
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid)); /* see above */
        asm volatile("" : "+v"(tid));

        T gy[R][nq], wy[R][nq], wz[R][nq];

        /* F1 [z-lines (i, j)]: gather p from the window, interpolate along z
         * -> TA at i + n j + n^2 qz */
#pragma unroll
        for (int rr = 0; rr < RA; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlA) {
                int nodexy, oz1;
                if constexpr (QX) {
                    const int c = l / n2, rem = l % n2, i = rem % n, j = rem / n;
                    const int cy = dTX.div(c), cx = c - cy * TXa;
                    nodexy = cx * K + i + PW * (cy * K + j);
                    oz1 = c * CS + rem;
                } else {
                    nodexy = oW[rr];
                    oz1 = oZ[rr];
                }
                T u[n];
#pragma unroll
                for (int z = 0; z < n; ++z) {
                    int slot = s0 + z;
                    if (slot > K) slot -= K + 1;
                    u[z] = win[slot * PNM + nodexy];
                }
#pragma unroll
                for (int q = 0; q < nq; ++q) TA[oz1 + n2 * q] = GLLQ ? u[q] : row_dot(cS, q, u);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* F2 [x-lines (j, qz)]: interpolate along x -> TB at qx + nq j + nq n qz */
#pragma unroll
        for (int rr = 0; rr < RB && !GLLQ; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlB) {
                int base, bout;
                if constexpr (QX) {
                    const int c = l / nnq, rem = l % nnq;
                    base = c * CS + n * rem;
                    bout = c * CS + nq * rem;
                } else {
                    base = bout = oX[rr];
                }
                T u[n];
#pragma unroll
                for (int i = 0; i < n; ++i) u[i] = TA[base + i];
#pragma unroll
                for (int q = 0; q < nq; ++q) TB[bout + q] = row_dot(cS, q, u);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* F3 [y-lines (qx, qz)]: interpolate along y -> values at the Gauss
         * points in TA at qx + nq qy + nq^2 qz, y derivative kept in registers */
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                int base, bin;
                if constexpr (QX) {
                    const int c = l / q2, rem = l % q2, i = rem % nq, z = rem / nq;
                    base = c * CS + i + q2 * z;
                    bin = c * CS + i + nnq * z;
                } else {
                    base = bin = oY[rr];
                }
                T u[n], uq[nq];
#pragma unroll
                for (int j = 0; j < n; ++j) u[j] = GLLQ ? TA[base + nq * j] : TB[bin + nq * j];
#pragma unroll
                for (int q = 0; q < nq; ++q) {
                    if (GLLQ) {
                        uq[q] = u[q]; /* values already in TA */
                    } else {
                        uq[q] = row_dot(cS, q, u);
                        TA[base + nq * q] = uq[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < nq && !MASS; ++q) gy[rr][q] = row_dot(cD, q, uq);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* G of this layer: loads issued here, consumed after the x and z
         * derivative passes */
        if (GPF == 1) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int l = tid + WG * rr;
#pragma unroll
                for (int j = 0; j < nq; ++j)
#pragma unroll
                    for (int c = 0; c < NG; ++c) gp[rr][c][j] = (l < nlines) ? gload<NTG>(&Gl[c * gcomp + j * gq + l]) : (T)0;
            }
        }
        /* F4 [x-lines (qy, qz)]: x derivative */
#pragma unroll
        for (int rr = 0; rr < R && !MASS; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                const int base = QX ? (l / q2) * CS + nq * (l % q2) : oX[rr];
                T u[nq];
#pragma unroll
                for (int i = 0; i < nq; ++i) u[i] = TA[base + i];
#pragma unroll
                for (int q = 0; q < nq; ++q) TB[base + q] = row_dot(cD, q, u);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* F5 [z-lines (qx, qy)]: z derivative, in place */
#pragma unroll
        for (int rr = 0; rr < R && !MASS; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                const int base = QX ? (l / q2) * CS + (l % q2) : oZ[rr];
                T u[nq];
#pragma unroll
                for (int z = 0; z < nq; ++z) u[z] = TA[base + q2 * z];
#pragma unroll
                for (int q = 0; q < nq; ++q) TA[base + q2 * q] = row_dot(cD, q, u);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* G [y-lines (qx, qz)]: flux = G_q grad u at each Gauss point; y part
         * of the transposed derivative in registers.  Mass operator: the
         * values scaled by a_e w_q det J_q, into TB. */
#pragma unroll
        for (int rr = 0; rr < R && MASS && !QGEOM; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                const int base = QX ? (l / q2) * CS + (l % q2) % nq + q2 * ((l % q2) / nq) : oY[rr];
                if (!GPF) {
#pragma unroll
                    for (int j = 0; j < nq; ++j) gp[rr][0][j] = gload<NTG>(&Gl[j * gq + l]);
                    /* every load of the line is issued before the first use */
                    asm volatile("" ::: "memory");
                }
#pragma unroll
                for (int j = 0; j < nq; ++j) TB[base + nq * j] = gp[rr][0][j] * TA[base + nq * j];
            }
        }
#pragma unroll
        for (int rr = 0; rr < R && QGEOM; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                const int c = l / q2, rem = l % q2, i = rem % nq, z = rem / nq;
                const int base = c * CS + i + q2 * z;
                /* this line's Gauss coordinates and weights in x and z */
                T tx = 0, tz = 0, wx = 0, wz = 0;
#pragma unroll
                for (int m = 0; m < nq; ++m) {
                    tx = i == m ? cxq(m) : tx;
                    wx = i == m ? cwq(m) : wx;
                    tz = z == m ? cxq(m) : tz;
                    wz = z == m ? cwq(m) : wz;
                }
                /* quadratic Lagrange basis on {0, 1/2, 1} and its derivative */
                const T Nx[3] = {(2 * tx - 1) * (tx - 1), 4 * tx * (1 - tx), tx * (2 * tx - 1)};
                const T dNx[3] = {4 * tx - 3, 4 - 8 * tx, 4 * tx - 1};
                const T Nz[3] = {(2 * tz - 1) * (tz - 1), 4 * tz * (1 - tz), tz * (2 * tz - 1)};
                const T dNz[3] = {4 * tz - 3, 4 - 8 * tz, 4 * tz - 1};
                /* the geometry contracted in x and z for this line:
                 * V = sum N_a N_d x, Vx = sum N_a' N_d x, Vz = sum N_a N_d' x,
                 * per component and y point b */
                const T *Xc = XS + c * QGEOM_STRIDE;
                T V[3][3], Vx[3][3], Vz[3][3];
#pragma unroll
                for (int co = 0; co < 3; ++co)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        T v = 0, vx = 0, vz = 0;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const T x0 = Xc[co * 27 + 9 * d + 3 * b], x1 = Xc[co * 27 + 9 * d + 3 * b + 1],
                                    x2 = Xc[co * 27 + 9 * d + 3 * b + 2];
                            const T sv = Nx[0] * x0 + Nx[1] * x1 + Nx[2] * x2;
                            const T sx = dNx[0] * x0 + dNx[1] * x1 + dNx[2] * x2;
                            v += Nz[d] * sv;
                            vz += dNz[d] * sv;
                            vx += Nz[d] * sx;
                        }
                        V[co][b] = v;
                        Vx[co][b] = vx;
                        Vz[co][b] = vz;
                    }
                const T aw = Xc[81] * wx * wz;
                T fy[nq];
#pragma unroll
                for (int j = 0; j < nq; ++j) {
                    const T ty = cxq(j);
                    const T Ny[3] = {(2 * ty - 1) * (ty - 1), 4 * ty * (1 - ty), ty * (2 * ty - 1)};
                    const T dNy[3] = {4 * ty - 3, 4 - 8 * ty, 4 * ty - 1};
                    T J[3][3];
#pragma unroll
                    for (int co = 0; co < 3; ++co) {
                        J[co][0] = Vx[co][0] * Ny[0] + Vx[co][1] * Ny[1] + Vx[co][2] * Ny[2];
                        J[co][1] = V[co][0] * dNy[0] + V[co][1] * dNy[1] + V[co][2] * dNy[2];
                        J[co][2] = Vz[co][0] * Ny[0] + Vz[co][1] * Ny[1] + Vz[co][2] * Ny[2];
                    }
                    if (MASS) {
                        /* a_e w_q det J_q times the value at the point */
                        const T det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) +
                                      J[0][1] * (J[1][2] * J[2][0] - J[1][0] * J[2][2]) +
                                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                        TB[base + nq * j] = aw * cwq(j) * det * TA[base + nq * j];
                        continue;
                    }
                    /* adjugate (det J times J^{-1}) and determinant */
                    const T A00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], A01 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
                            A02 = J[0][1] * J[1][2] - J[0][2] * J[1][1], A10 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
                            A11 = J[0][0] * J[2][2] - J[0][2] * J[2][0], A12 = J[0][2] * J[1][0] - J[0][0] * J[1][2],
                            A20 = J[1][0] * J[2][1] - J[1][1] * J[2][0], A21 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
                            A22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                    const T det = J[0][0] * A00 + J[0][1] * A10 + J[0][2] * A20;
                    /* flux a_e w_q det J J^{-1} J^{-T} grad u = sc A (A^T grad u)
                     * with sc = a_e w_q / det J, without forming the tensor */
                    const T sc = aw * cwq(j) / det;
                    const T ux = TB[base + nq * j], uy = gy[rr][j], uz = TA[base + nq * j];
                    const T t0 = A00 * ux + A10 * uy + A20 * uz, t1 = A01 * ux + A11 * uy + A21 * uz,
                            t2 = A02 * ux + A12 * uy + A22 * uz;
                    const T fx = sc * (A00 * t0 + A01 * t1 + A02 * t2);
                    fy[j] = sc * (A10 * t0 + A11 * t1 + A12 * t2);
                    const T fz = sc * (A20 * t0 + A21 * t1 + A22 * t2);
                    TB[base + nq * j] = fx;
                    TA[base + nq * j] = fz;
                }
#pragma unroll
                for (int m = 0; m < nq && !MASS; ++m) wy[rr][m] = col_dot(cD, m, fy);
            }
        }
#pragma unroll
        for (int rr = 0; rr < R && !MASS && !QGEOM; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                const int base = QX ? (l / q2) * CS + (l % q2) % nq + q2 * ((l % q2) / nq) : oY[rr];
                T fy[nq];
#pragma unroll
                for (int j = 0; j < nq; ++j) {
                    if (!GPF) {
#pragma unroll
                        for (int c2 = 0; c2 < 6; ++c2) gp[rr][c2][j] = gload<NTG>(&Gl[c2 * gcomp + j * gq + l]);
                    }
                    const T ux = TB[base + nq * j], uy = gy[rr][j], uz = TA[base + nq * j];
                    const T fx = gp[rr][0][j] * ux + gp[rr][3][j] * uy + gp[rr][4][j] * uz;
                    fy[j] = gp[rr][3][j] * ux + gp[rr][1][j] * uy + gp[rr][5][j] * uz;
                    const T fz = gp[rr][4][j] * ux + gp[rr][5][j] * uy + gp[rr][2][j] * uz;
                    TB[base + nq * j] = fx;
                    TA[base + nq * j] = fz;
                }
#pragma unroll
                for (int m = 0; m < nq; ++m) wy[rr][m] = col_dot(cD, m, fy);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* B2 [x-lines (qy, qz)]: transposed x derivative, in place; B3
         * [z-lines (qx, qy)]: transposed z derivative into registers */
#pragma unroll
        for (int rr = 0; rr < R && !MASS; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                {
                    const int base = QX ? (l / q2) * CS + nq * (l % q2) : oX[rr];
                    T f[nq];
#pragma unroll
                    for (int q = 0; q < nq; ++q) f[q] = TB[base + q];
#pragma unroll
                    for (int m = 0; m < nq; ++m) TB[base + m] = col_dot(cD, m, f);
                }
                {
                    const int base = QX ? (l / q2) * CS + (l % q2) : oZ[rr];
                    T f[nq];
#pragma unroll
                    for (int q = 0; q < nq; ++q) f[q] = TA[base + q2 * q];
#pragma unroll
                    for (int m = 0; m < nq; ++m) wz[rr][m] = col_dot(cD, m, f);
                }
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* B4 [y-lines (qx, qz)]: add the y part */
#pragma unroll
        for (int rr = 0; rr < R && !MASS; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                const int base = QX ? (l / q2) * CS + (l % q2) % nq + q2 * ((l % q2) / nq) : oY[rr];
#pragma unroll
                for (int j = 0; j < nq; ++j) TB[base + nq * j] += wy[rr][j];
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* B5 [z-lines (qx, qy)]: add the z part, transposed interpolation
         * along z -> qx + nq qy + nq^2 z */
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlines) {
                const int base = QX ? (l / q2) * CS + (l % q2) : oZ[rr];
                T w[nq];
#pragma unroll
                for (int q = 0; q < nq; ++q) w[q] = MASS ? TB[base + q2 * q] : TB[base + q2 * q] + wz[rr][q];
#pragma unroll
                for (int z = 0; z < n; ++z) TB[base + q2 * z] = GLLQ ? w[z] : col_dot(cS, z, w);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* B6 [x-lines (qy, z)]: transposed interpolation along x -> i + nq qy + nq^2 z */
#pragma unroll
        for (int rr = 0; rr < RB && !GLLQ; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlB) {
                const int base = QX ? (l / nnq) * CS + nq * (l % nnq) : oX[rr];
                T w[nq];
#pragma unroll
                for (int q = 0; q < nq; ++q) w[q] = TB[base + q];
#pragma unroll
                for (int i = 0; i < n; ++i) TB[base + i] = col_dot(cS, i, w);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
        /* B7 [y-lines (i, z)]: transposed interpolation along y -> cell
         * vectors at i + nq j + nq^2 z */
#pragma unroll
        for (int rr = 0; rr < RA && !GLLQ; ++rr) {
            const int l = tid + WG * rr;
            if (l < nlA) {
                const int base = QX ? (l / n2) * CS + (l % n2) % n + q2 * ((l % n2) / n) : oY[rr];
                T w[nq];
#pragma unroll
                for (int q = 0; q < nq; ++q) w[q] = TB[base + nq * q];
#pragma unroll
                for (int j = 0; j < n; ++j) TB[base + nq * j] = col_dot(cS, j, w);
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));

        /* ---- sum over cells and post ---- */
        /* the CG post of a tile-interior node at vector index i (fast path) */
        auto post_fast = [&](int64_t i, int node, int slot, T v, bool reg, T rk, T dk) {
            if (MODE == MODE_VMULT) {
                a.dst[i] = v;
            } else {
                const T rn = reg ? rk : a.r[i];
                const T dv = MODE == MODE_CG_NOPREC ? (T)1 : (reg ? dk : a.dinv[i]);
                const T pn = win[slot * PNM + node];
                const T zr = dv * rn, zv = dv * v;
                acc[0] += rn * rn;
                acc[1] += pn * v;
                acc[2] += rn * v;
                acc[3] += v * v;
                acc[4] += rn * zr;
                acc[5] += rn * zv;
                acc[6] += v * zv;
                a.v[i] = v;
            }
        };
        /* plane z = 0 of the layer (plane L K), completing the carry of the
         * layer below: interior nodes (fast path, L > 0; their pre ran in
         * the layer below, so r and D^{-1} are re-read) */
        if (L > 0 && fast) {
            const int64_t fb0 = vb13 + (int64_t)(L * K - 1) * SXY;
#pragma unroll
            for (int c = 0; c < NF0; ++c) {
                const int f = tid + WG * c;
                if (f < SXY) {
                    const int node = inode(f);
                    const T v = cv[(L & 1) * PNM + node] + sum_cells(desc[node], 0);
                    post_fast(fb0 + f, node, s0, v, false, (T)0, (T)0);
                }
            }
        }
        /* plane z = 0, general path: the whole plane in the first layer (the
         * tile's bottom plane), else its ring */
        {
            const bool whole = L == 0 || !fast;
            const int N0 = whole ? PN : NRING;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int f = tid + WG * c;
                if (f < N0) {
                    const int node = whole ? f : ring[f];
                    const int4 dsc = desc[node];
                    T v = sum_cells(dsc, 0);
                    if (L > 0) v = cv[(L & 1) * PNM + node] + v;
                    post_node(dsc, node, L * K, s0, v, false, (T)0, (T)0);
                }
            }
        }
        /* planes z = 1..K; the top plane is carried unless it is the tile's
         * last.  Fast path in the thread mapping of its pre. */
#pragma unroll
        for (int s = 0; s < NFI; ++s) {
            const int f = tid + WG * s;
            if (f < nf) {
                const int zq = dSXY.div(f), node = inode(f - zq * SXY), zl = 1 + zq;
                const T v = sum_cells(desc[node], zl);
                if (zl == K && L + 1 < TZa) {
                    cv[((L + 1) & 1) * PNM + node] = v;
                } else {
                    int slot = s0 + zl;
                    if (slot > K) slot -= K + 1;
                    post_fast(fb + f, node, slot, v, CARRYF, kr[s], kd[s]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int f = tid + WG * s;
            if (f < NR) {
                int zl, node;
                gdecode(f, zl, node);
                const int4 dsc = desc[node];
                const T v = sum_cells(dsc, zl);
                if (zl == K && L + 1 < TZa) {
                    cv[((L + 1) & 1) * PNM + node] = v;
                } else {
                    int slot = s0 + zl;
                    if (slot > K) slot -= K + 1;
                    post_node(dsc, node, L * K + zl, slot, v, false, (T)0, (T)0);
                }
            }
        }
        if (FLUSH) {
            /* fixed order: shuffle tree in the wave, then the wave's slot in
             * layer order */
            const int lane = tid0 & 63, wave = tid0 >> 6;
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                T sv = acc[c];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) sv += __shfl_xor(sv, off, 64);
                if (lane == 0) wacc[wave * 8 + c] += sv;
                acc[c] = 0;
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tid));
    }

    if (FLUSH) {
        if (tid0 < 7) {
            T sv = 0;
            for (int w = 0; w < WG / 64; ++w) sv += wacc[w * 8 + tid0];
            a.dots[tile * 8 + tid0] = sv;
        }
    } else if (mode_is_cg(MODE)) {
        block_reduce<T, 7, WG>(acc, red, a.dots + tile * 8);
    }
}

template <int K, typename T, int MODE, int OPV = OPV_LAPLACE, int QX = 0>
__global__ __launch_bounds__(Cfg<K>::WG)
__attribute__((amdgpu_waves_per_eu(MFCG_WPE_MIN_Q(K, QX, OPV), 8)))
void fused_tile_kernel(const IterArgs<T> a)
{
    if (mode_is_cg(MODE) && a.st->flag != FLAG_RUN) return;
    fused_tile<K, T, MODE, OPV, true, QX>(a, xcd_remap(blockIdx.x, gridDim.x));
}

/* Several vectors on one operator: one launch over (tile, component)
 * pairs, the component fastest, so the workgroups of one tile's m
 * components are dispatched together on one XCD and the geometry tensor
 * they all apply is fetched from HBM about once and then served from that
 * XCD's L2.  Component c works on the vectors at offset c*nstride, its
 * shared-node partial sums at c*pstride, its inner-product records at
 * c*dstride and the CG state at a.st + c*sstride: sstride = 0 for the
 * vector problem (three components, one CG), 1 for independent right-hand
 * sides (one CG each; a component whose CG has stopped is skipped). */
template <int K, int MODE, int OPV, int QX = 0>
__global__ __launch_bounds__(Cfg<K>::WG)
__attribute__((amdgpu_waves_per_eu(MFCG_WPE_MIN_Q(K, QX, OPV), 8)))
void fused_tile_vec_kernel(const IterArgs<double> a, int m, int64_t nstride, int64_t pstride, int64_t dstride,
                           int sstride)
{
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int c = (int)(lb % m);
    if (a.st[c * sstride].flag != FLAG_RUN) return;
    IterArgs<double> b = a;
    b.st += c * sstride;
    b.r += c * nstride;
    b.p += c * nstride;
    b.v += c * nstride;
    b.x += c * nstride;
    b.part += c * pstride;
    b.dots += c * dstride;
    fused_tile<K, double, MODE, OPV, false, QX>(b, lb / m);
}

/* Batch of problems of degree K: one workgroup per (problem, tile) item of
 * the work list; problems that have left the running state are skipped. */
template <int K, typename T>
__global__ __launch_bounds__(Cfg<K>::WG)
__attribute__((amdgpu_waves_per_eu(MFCG_WPE_MIN_BATCH(K), 8)))
void fused_batch_kernel(const IterArgs<T> *__restrict__ probs, const int2 *__restrict__ items, int nitems)
{
    const int2 it = items[xcd_remap(blockIdx.x, nitems)];
    const int p = __builtin_amdgcn_readfirstlane(it.x);
    const int64_t tile = __builtin_amdgcn_readfirstlane(it.y);
    const IterArgsG<T> &a = *(const IterArgsG<T> *)(probs + p);
    if (a.st->flag != FLAG_RUN) return;
    fused_tile<K, T, MODE_CG>(a, tile);
}

/* ------------------------------------------------------------------ */
/* Launch wrappers of one degree                                       */
/* ------------------------------------------------------------------ */

template <int K, int OPV, int QX>
static inline void launch_fused_variant(int mode, dim3 grid, dim3 block, const IterArgs<double> &a, hipStream_t s)
{
    if (mode == MODE_CG)
        hipLaunchKernelGGL((fused_tile_kernel<K, double, MODE_CG, OPV, QX>), grid, block, 0, s, a);
    else if (mode == MODE_CG_NOPREC)
        hipLaunchKernelGGL((fused_tile_kernel<K, double, MODE_CG_NOPREC, OPV, QX>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((fused_tile_kernel<K, double, MODE_VMULT, OPV, QX>), grid, block, 0, s, a);
}

template <int K, typename T>
static inline hipError_t launch_fused_k(int mode, const IterArgs<T> &a, hipStream_t s)
{
    dim3 grid((unsigned)a.L.ntiles), block(Cfg<K>::WG);
    if (mode & (MODE_GLL | MODE_MASS | MODE_Q2 | MODE_QGEOM)) {
        if constexpr (!std::is_same<T, double>::value) {
            return hipErrorInvalidValue; /* FP64 only */
        } else {
            const bool mass = mode & MODE_MASS, gll = mode & MODE_GLL, q2 = mode & MODE_Q2, qg = mode & MODE_QGEOM;
            if (gll && (mass || q2)) return hipErrorInvalidValue;
            if (qg && gll) return hipErrorInvalidValue;
            mode &= ~(MODE_GLL | MODE_MASS | MODE_Q2 | MODE_QGEOM);
            if (mode != MODE_CG && mode != MODE_CG_NOPREC && mode != MODE_VMULT) return hipErrorInvalidValue;
            if (qg && q2) {
                if constexpr (K <= 7) {
                    if (mass) launch_fused_variant<K, OPV_MASS_QGEOM, 1>(mode, grid, block, a, s);
                    else launch_fused_variant<K, OPV_LAPLACE_QGEOM, 1>(mode, grid, block, a, s);
                } else {
                    return hipErrorInvalidValue;
                }
            } else if (qg) {
                if (mass) launch_fused_variant<K, OPV_MASS_QGEOM, 0>(mode, grid, block, a, s);
                else launch_fused_variant<K, OPV_LAPLACE_QGEOM, 0>(mode, grid, block, a, s);
            } else if (q2) {
                if constexpr (K <= 7) {
                    if (mass) launch_fused_variant<K, OPV_MASS, 1>(mode, grid, block, a, s);
                    else launch_fused_variant<K, OPV_LAPLACE, 1>(mode, grid, block, a, s);
                } else {
                    return hipErrorInvalidValue;
                }
            } else if (mass) {
                launch_fused_variant<K, OPV_MASS, 0>(mode, grid, block, a, s);
            } else {
                launch_fused_variant<K, OPV_LAPLACE_GLL, 0>(mode, grid, block, a, s);
            }
            return hipGetLastError();
        }
    }
    if (mode == MODE_CG) {
        hipLaunchKernelGGL((fused_tile_kernel<K, T, MODE_CG>), grid, block, 0, s, a);
    } else if (mode == MODE_CG_NOPREC) {
        if constexpr (!std::is_same<T, double>::value) return hipErrorInvalidValue; /* FP64 only */
        else hipLaunchKernelGGL((fused_tile_kernel<K, T, MODE_CG_NOPREC>), grid, block, 0, s, a);
    } else {
        hipLaunchKernelGGL((fused_tile_kernel<K, T, MODE_VMULT>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int K>
static inline hipError_t launch_fused_vec_k(int mode, const IterArgs<double> &a, int m, int64_t nstride,
                                            int64_t pstride, int64_t dstride, int sstride, hipStream_t s)
{
    dim3 grid((unsigned)(m * a.L.ntiles)), block(Cfg<K>::WG);
    if (mode == (MODE_CG | MODE_Q2) || mode == (MODE_CG | MODE_MASS | MODE_Q2) || mode == (MODE_CG | MODE_QGEOM | MODE_Q2) ||
        mode == (MODE_CG | MODE_QGEOM | MODE_MASS | MODE_Q2)) {
        if constexpr (K <= 7) {
            if ((mode & MODE_QGEOM) && (mode & MODE_MASS))
                hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_MASS_QGEOM, 1>), grid, block, 0, s, a, m,
                                   nstride, pstride, dstride, sstride);
            else if (mode & MODE_QGEOM)
                hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_LAPLACE_QGEOM, 1>), grid, block, 0, s, a, m,
                                   nstride, pstride, dstride, sstride);
            else if (mode & MODE_MASS)
                hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_MASS, 1>), grid, block, 0, s, a, m, nstride,
                                   pstride, dstride, sstride);
            else
                hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_LAPLACE, 1>), grid, block, 0, s, a, m, nstride,
                                   pstride, dstride, sstride);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (mode == MODE_CG)
        hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_LAPLACE>), grid, block, 0, s, a, m, nstride, pstride,
                           dstride, sstride);
    else if (mode == (MODE_CG | MODE_GLL))
        hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_LAPLACE_GLL>), grid, block, 0, s, a, m, nstride, pstride,
                           dstride, sstride);
    else if (mode == (MODE_CG | MODE_MASS))
        hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_MASS>), grid, block, 0, s, a, m, nstride, pstride,
                           dstride, sstride);
    else if (mode == (MODE_CG | MODE_QGEOM | MODE_MASS))
        hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_MASS_QGEOM>), grid, block, 0, s, a, m, nstride,
                           pstride, dstride, sstride);
    else if (mode == (MODE_CG | MODE_QGEOM))
        hipLaunchKernelGGL((fused_tile_vec_kernel<K, MODE_CG, OPV_LAPLACE_QGEOM>), grid, block, 0, s, a, m, nstride,
                           pstride, dstride, sstride);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}


/* ------------------------------------------------------------------ */
/* Per-degree entry points (defined in fused_k<K>.hip)                 */
/* ------------------------------------------------------------------ */

template <int K>
struct FusedDeg {
    static hipError_t fused64(int mode, const IterArgs<double> &a, hipStream_t s);
    static hipError_t fused32(int mode, const IterArgs<float> &a, hipStream_t s);
    static hipError_t vec(int mode, const IterArgs<double> &a, int m, int64_t nstride, int64_t pstride,
                          int64_t dstride, int sstride, hipStream_t s);
    static void batch(const IterArgs<double> *probs, const int2 *items, int nitems, hipStream_t s);
};

/* The definitions of one degree's entry points (one translation unit per
 * degree, so that the degrees compile in parallel). */
#define MFCG_FUSED_DEGREE(K)                                                                                         \
    template <>                                                                                                       \
    hipError_t FusedDeg<K>::fused64(int mode, const IterArgs<double> &a, hipStream_t s)                               \
    {                                                                                                                 \
        return launch_fused_k<K, double>(mode, a, s);                                                                 \
    }                                                                                                                 \
    template <>                                                                                                       \
    hipError_t FusedDeg<K>::fused32(int mode, const IterArgs<float> &a, hipStream_t s)                                \
    {                                                                                                                 \
        return launch_fused_k<K, float>(mode, a, s);                                                                  \
    }                                                                                                                 \
    template <>                                                                                                       \
    hipError_t FusedDeg<K>::vec(int mode, const IterArgs<double> &a, int m, int64_t nstride, int64_t pstride,         \
                                int64_t dstride, int sstride, hipStream_t s)                                          \
    {                                                                                                                 \
        return launch_fused_vec_k<K>(mode, a, m, nstride, pstride, dstride, sstride, s);                              \
    }                                                                                                                 \
    template <>                                                                                                       \
    void FusedDeg<K>::batch(const IterArgs<double> *probs, const int2 *items, int nitems, hipStream_t s)              \
    {                                                                                                                 \
        hipLaunchKernelGGL((fused_batch_kernel<K, double>), dim3((unsigned)nitems), dim3(Cfg<K>::WG), 0, s, probs,    \
                           items, nitems);                                                                            \
    }

}  // namespace mfcg
