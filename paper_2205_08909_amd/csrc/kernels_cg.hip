/*
 * kernels_cg.hip -- the per-iteration kernels of the fused Jacobi-PCG
 * (Algorithm 5 of Kronbichler, Sashko, Munch, with the vector updates and
 * inner products embedded in the cell loop of the matrix-free operator,
 * Sec. 5), written for gfx950 (wave64, 160 KB LDS per CU).
 *
 * One iteration k is three launches:
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
 *           of k+1 node planes.
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
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fused_tile.h"

namespace mfcg {

void tile_limits(int K, int *tx, int *ty) { tile_limits_impl(K, tx, ty); }
int fused_block_size(int K) { return fused_block_size_impl(K); }

/* ------------------------------------------------------------------ */
/* Shared-node kernel with the single-pass finish                      */
/* ------------------------------------------------------------------ */

/* nodes per thread of the shared-node kernel, processed with their loads
 * issued together */
constexpr int SH_UNROLL = 4;

/* Block blk of nblk of one problem's shared-node pass. */
template <typename T, int MODE, typename ARGS>
__device__ __forceinline__ void shared_nodes(const ARGS &a, const int blk, const int nblk, T *red)
{
    const auto &L = a.L;

    T alpha = 0, beta = 0, ratio = 0;
    bool xupd = false;
    if (mode_is_cg(MODE)) {
        alpha = (T)a.st->alpha;
        beta = (T)a.st->beta;
        ratio = (T)a.st->ratio;
        const int kk = a.st->k + 1;
        xupd = (kk > 1) && (kk & 1);
    }
    T acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = 0;

    const int64_t stride = (int64_t)nblk * SHARED_WG;
    for (int64_t i0 = L.offF + (int64_t)blk * SHARED_WG + threadIdx.x; i0 < L.n; i0 += SH_UNROLL * stride) {
        T vs[SH_UNROLL], r0[SH_UNROLL], v0[SH_UNROLL], p0[SH_UNROLL], dv[SH_UNROLL], x0[SH_UNROLL];
        bool ok[SH_UNROLL], cons[SH_UNROLL];
#pragma unroll
        for (int u = 0; u < SH_UNROLL; ++u) {
            const int64_t i = i0 + u * stride;
            ok[u] = i < L.n;
            cons[u] = i >= L.offC;
            T v = 0;
            if (ok[u]) {
                if (i < L.offE) {
                    const int64_t j = i - L.offF;
                    v = a.part[L.partF + j] + a.part[L.partF + L.nF + j];
                } else if (i < L.offV) {
                    const T *q = a.part + L.partE + (i - L.offE);
                    v = ((q[0] + q[L.nE]) + q[2 * L.nE]) + q[3 * L.nE];
                } else if (i < L.offC) {
                    const T *q = a.part + L.partV + (i - L.offV);
                    v = q[0];
#pragma unroll
                    for (int s = 1; s < 8; ++s) v += q[s * L.nV];
                }
                if (mode_is_cg(MODE)) {
                    r0[u] = a.r[i];
                    v0[u] = a.v[i];
                    p0[u] = a.p[i];
                    dv[u] = MODE == MODE_CG_NOPREC ? (T)1 : a.dinv[i];
                    x0[u] = xupd ? a.x[i] : (T)0;
                } else if (cons[u]) {
                    v = a.src[i];
                }
            }
            vs[u] = v;
        }
#pragma unroll
        for (int u = 0; u < SH_UNROLL; ++u) {
            if (!ok[u]) continue;
            const int64_t i = i0 + u * stride;
            if (MODE == MODE_VMULT) {
                a.dst[i] = vs[u];
                continue;
            }
            T rn, pn;
            pre_update(r0[u], v0[u], p0[u], dv[u], alpha, beta, rn, pn);
            if (xupd) a.x[i] = x_update(x0[u], r0[u], p0[u], dv[u], alpha, ratio);
            const T v = cons[u] ? pn : vs[u]; /* identity rows on Dirichlet nodes */
            a.r[i] = rn;
            a.p[i] = pn;
            a.v[i] = v;
            const T zr = dv[u] * rn, zv = dv[u] * v;
            acc[0] += rn * rn;
            acc[1] += pn * v;
            acc[2] += rn * v;
            acc[3] += v * v;
            acc[4] += rn * zr;
            acc[5] += rn * zv;
            acc[6] += v * zv;
        }
    }
    if (MODE == MODE_VMULT) return;

    block_reduce<T, 7, SHARED_WG>(acc, red, a.dots + (L.ntiles + blk) * 8);
}

template <typename T, int MODE>
__global__ __launch_bounds__(SHARED_WG) void shared_node_kernel(const IterArgs<T> a)
{
    __shared__ T red[8 * (SHARED_WG / 64)];
    if (mode_is_cg(MODE) && a.st->flag != FLAG_RUN) return;
    shared_nodes<T, MODE>(a, blockIdx.x, gridDim.x, red);
}

/* Batch: one workgroup per (problem, block) item. */
template <typename T>
__global__ __launch_bounds__(SHARED_WG) void shared_batch_kernel(const IterArgs<T> *__restrict__ probs,
                                                                 const int2 *__restrict__ items)
{
    __shared__ T red[8 * (SHARED_WG / 64)];
    const int2 it = items[blockIdx.x];
    const int p = __builtin_amdgcn_readfirstlane(it.x);
    const IterArgsG<T> &a = *(const IterArgsG<T> *)(probs + p);
    if (a.st->flag != FLAG_RUN) return;
    shared_nodes<T, MODE_CG>(a, __builtin_amdgcn_readfirstlane(it.y), a.nshared_blocks, red);
}

/* One block: the seven inner products of the iteration from all per-block
 * partials of the two kernels above (fixed order), then alpha, beta and the
 * convergence test of Algorithm 5 into the device state.  A separate launch
 * makes every partial visible without a device-wide cache write-back in
 * each block of the shared-node kernel. */
template <typename T>
__global__ __launch_bounds__(SHARED_WG) void finish_kernel(const IterArgs<T> a)
{
    __shared__ T red[8 * (SHARED_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    finish_iteration<T>(a, a.L.ntiles + a.nshared_blocks, red);
}

/* The same over an explicit record count (vector problems: every
 * component's records in a row). */
__global__ __launch_bounds__(SHARED_WG) void finish_parts_kernel(const IterArgs<double> a, int64_t nparts)
{
    __shared__ double red[8 * (SHARED_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    finish_iteration<double>(a, nparts, red);
}

/* Independent right-hand sides on one operator: blockIdx.y is the
 * right-hand side c, whose vectors, shared-node partial sums, records and
 * CG state sit at c*nstride, c*pstride, c*dstride and a.st + c. */
__global__ __launch_bounds__(SHARED_WG) void shared_node_multi_kernel(const IterArgs<double> a, int64_t nstride,
                                                                      int64_t pstride, int64_t dstride)
{
    __shared__ double red[8 * (SHARED_WG / 64)];
    const int c = blockIdx.y;
    if (a.st[c].flag != FLAG_RUN) return;
    IterArgs<double> b = a;
    b.r += c * nstride;
    b.p += c * nstride;
    b.v += c * nstride;
    b.x += c * nstride;
    b.part += c * pstride;
    b.dots += c * dstride;
    b.st += c;
    shared_nodes<double, MODE_CG>(b, blockIdx.x, gridDim.x, red);
}

/* One block per right-hand side: its records, its scalars, its history
 * (c*hstride). */
__global__ __launch_bounds__(SHARED_WG) void finish_multi_kernel(const IterArgs<double> a, int64_t dstride,
                                                                 int64_t hstride)
{
    __shared__ double red[8 * (SHARED_WG / 64)];
    const int c = blockIdx.x;
    if (a.st[c].flag != FLAG_RUN) return;
    IterArgs<double> b = a;
    b.dots += c * dstride;
    b.st += c;
    b.hist += c * hstride;
    finish_iteration<double>(b, a.L.ntiles + a.nshared_blocks, red);
}

/* Batch: one block per listed problem. */
template <typename T>
__global__ __launch_bounds__(SHARED_WG) void finish_batch_kernel(const IterArgs<T> *__restrict__ probs,
                                                                 const int *__restrict__ plist)
{
    __shared__ T red[8 * (SHARED_WG / 64)];
    const IterArgsG<T> &a = *(const IterArgsG<T> *)(probs + __builtin_amdgcn_readfirstlane(plist[blockIdx.x]));
    if (a.st->flag != FLAG_RUN) return;
    finish_iteration<T>(a, a.L.ntiles + a.nshared_blocks, red);
}

/* ------------------------------------------------------------------ */
/* Launch wrappers                                                     */
/* ------------------------------------------------------------------ */

template <typename T>
hipError_t launch_fused(int K, int mode, const IterArgs<T> &a, hipStream_t s)
{
    constexpr bool D = std::is_same<T, double>::value;
    auto pick = [&](auto deg) -> hipError_t {
        using F = decltype(deg);
        if constexpr (D) return F::fused64(mode, a, s);
        else return F::fused32(mode, a, s);
    };
    switch (K) {
    case 1: return pick(FusedDeg<1>{});
    case 2: return pick(FusedDeg<2>{});
    case 3: return pick(FusedDeg<3>{});
    case 4: return pick(FusedDeg<4>{});
    case 5: return pick(FusedDeg<5>{});
    case 6: return pick(FusedDeg<6>{});
    case 7: return pick(FusedDeg<7>{});
    case 8: return pick(FusedDeg<8>{});
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_shared(int mode, const IterArgs<T> &a, hipStream_t s)
{
    dim3 grid((unsigned)a.nshared_blocks), block(SHARED_WG);
    if (mode == MODE_CG) {
        hipLaunchKernelGGL((shared_node_kernel<T, MODE_CG>), grid, block, 0, s, a);
        hipLaunchKernelGGL((finish_kernel<T>), dim3(1), block, 0, s, a);
    } else if (mode == MODE_CG_NOPREC) {
        if constexpr (!std::is_same<T, double>::value) return hipErrorInvalidValue;
        else {
            hipLaunchKernelGGL((shared_node_kernel<T, MODE_CG_NOPREC>), grid, block, 0, s, a);
            hipLaunchKernelGGL((finish_kernel<T>), dim3(1), block, 0, s, a);
        }
    } else {
        hipLaunchKernelGGL((shared_node_kernel<T, MODE_VMULT>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_fused_vec(int K, int mode, const IterArgs<double> &a, int m, int64_t nstride, int64_t pstride,
                            int64_t dstride, int sstride, hipStream_t s)
{
    switch (K) {
    case 1: return FusedDeg<1>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    case 2: return FusedDeg<2>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    case 3: return FusedDeg<3>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    case 4: return FusedDeg<4>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    case 5: return FusedDeg<5>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    case 6: return FusedDeg<6>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    case 7: return FusedDeg<7>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    case 8: return FusedDeg<8>::vec(mode, a, m, nstride, pstride, dstride, sstride, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_shared_nofinish(const IterArgs<double> &a, hipStream_t s)
{
    hipLaunchKernelGGL((shared_node_kernel<double, MODE_CG>), dim3((unsigned)a.nshared_blocks), dim3(SHARED_WG), 0, s,
                       a);
    return hipGetLastError();
}

hipError_t launch_shared_finish_multi(const IterArgs<double> &a, int m, int64_t nstride, int64_t pstride,
                                      int64_t dstride, int64_t hstride, hipStream_t s)
{
    hipLaunchKernelGGL(shared_node_multi_kernel, dim3((unsigned)a.nshared_blocks, (unsigned)m), dim3(SHARED_WG), 0,
                       s, a, nstride, pstride, dstride);
    hipLaunchKernelGGL(finish_multi_kernel, dim3((unsigned)m), dim3(SHARED_WG), 0, s, a, dstride, hstride);
    return hipGetLastError();
}

__global__ void gather_states_kernel(const IterArgs<double> *__restrict__ probs, int np, CGState *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) out[i] = *probs[i].st;
}

hipError_t launch_gather_states(const IterArgs<double> *probs, int np, CGState *out, hipStream_t s)
{
    hipLaunchKernelGGL(gather_states_kernel, dim3((unsigned)((np + 63) / 64)), dim3(64), 0, s, probs, np, out);
    return hipGetLastError();
}

hipError_t launch_finish_parts(const IterArgs<double> &a, int64_t nparts, hipStream_t s)
{
    hipLaunchKernelGGL(finish_parts_kernel, dim3(1), dim3(SHARED_WG), 0, s, a, nparts);
    return hipGetLastError();
}

hipError_t launch_batch_iteration(const BatchLaunch &b, hipStream_t s)
{
    for (int K = 1; K <= 8; ++K) {
        const int ni = b.nitems[K];
        if (ni == 0) continue;
        switch (K) {
        case 1: FusedDeg<1>::batch(b.probs, b.items[K], ni, s); break;
        case 2: FusedDeg<2>::batch(b.probs, b.items[K], ni, s); break;
        case 3: FusedDeg<3>::batch(b.probs, b.items[K], ni, s); break;
        case 4: FusedDeg<4>::batch(b.probs, b.items[K], ni, s); break;
        case 5: FusedDeg<5>::batch(b.probs, b.items[K], ni, s); break;
        case 6: FusedDeg<6>::batch(b.probs, b.items[K], ni, s); break;
        case 7: FusedDeg<7>::batch(b.probs, b.items[K], ni, s); break;
        case 8: FusedDeg<8>::batch(b.probs, b.items[K], ni, s); break;
        }
    }
    if (b.nshared_items > 0)
        hipLaunchKernelGGL((shared_batch_kernel<double>), dim3((unsigned)b.nshared_items), dim3(SHARED_WG), 0, s,
                           b.probs, b.shared_items);
    if (b.nactive > 0)
        hipLaunchKernelGGL((finish_batch_kernel<double>), dim3((unsigned)b.nactive), dim3(SHARED_WG), 0, s, b.probs,
                           b.active);
    return hipGetLastError();
}

template hipError_t launch_fused<double>(int, int, const IterArgs<double> &, hipStream_t);
template hipError_t launch_fused<float>(int, int, const IterArgs<float> &, hipStream_t);
template hipError_t launch_shared<double>(int, const IterArgs<double> &, hipStream_t);
template hipError_t launch_shared<float>(int, const IterArgs<float> &, hipStream_t);

}  // namespace mfcg
