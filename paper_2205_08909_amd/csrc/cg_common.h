/*
 * cg_common.h -- device helpers shared by the fused CG kernels and the
 * unfused comparison solvers: the per-entry vector updates of Algorithm 5,
 * the deterministic block reduction, and the one-block finish that turns
 * the seven partial inner products into alpha_k, beta_k and the
 * convergence test (Algorithm 5, with the predicted residual norm
 * sqrt(gamma - 2 alpha b + alpha^2 c)).
 */
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "kernels.h"

namespace mfcg {

/* The batch kernels read each problem's arguments from device memory.
 * Pointers loaded from memory are generic to the compiler, which then
 * emits flat loads and stores: those count against the LDS wait counter
 * too, so every LDS wait also waits for them, and they cannot be scalar.
 * Read through these layout-identical views, whose pointers are declared
 * in the global address space, the same code compiles to global and scalar
 * memory instructions as it does for kernel arguments. */
/* (the host pass, which compiles no kernel code, sees plain pointers) */
#ifdef __HIP_DEVICE_COMPILE__
#define MFCG_GLOBAL __attribute__((address_space(1)))
#else
#define MFCG_GLOBAL
#endif
struct LayoutViewG {
    Dim1 d[3];
    int64_t n;
    int64_t nI, nF, nE, nV, nC;
    int64_t offF, offE, offV, offC;
    int64_t partF, partE, partV;
    int64_t ntiles;
    const MFCG_GLOBAL int64_t *ent_base;
    const MFCG_GLOBAL EntityRef *tile_ent;
    const MFCG_GLOBAL TileDesc *tiles;
};
template <typename T>
struct IterArgsG {
    LayoutViewG L;
    const MFCG_GLOBAL T *G;
    const MFCG_GLOBAL T *dinv;
    MFCG_GLOBAL T *r, *p, *v, *x;
    const MFCG_GLOBAL T *src;
    MFCG_GLOBAL T *dst;
    MFCG_GLOBAL T *part;
    MFCG_GLOBAL T *dots;
    MFCG_GLOBAL CGState *st;
    MFCG_GLOBAL double *hist;
    int32_t nshared_blocks;
};
static_assert(sizeof(LayoutViewG) == sizeof(LayoutView) && offsetof(LayoutViewG, tiles) == offsetof(LayoutView, tiles),
              "global view of LayoutView");
static_assert(sizeof(IterArgsG<double>) == sizeof(IterArgs<double>) &&
                  offsetof(IterArgsG<double>, G) == offsetof(IterArgs<double>, G) &&
                  offsetof(IterArgsG<double>, dots) == offsetof(IterArgs<double>, dots) &&
                  offsetof(IterArgsG<double>, nshared_blocks) == offsetof(IterArgs<double>, nshared_blocks),
              "global view of IterArgs");

}  // namespace mfcg

namespace mfcg {

constexpr int SHARED_WG = 256;

/* The "pre" update of one entry, shared by both kernels so that the value
 * a tile recomputes for a shared node is bitwise the value the shared-node
 * kernel stores. */
template <typename T>
__device__ __forceinline__ void pre_update(T r, T v, T p, T dinv, T alpha, T beta, T &rn, T &pn)
{
    rn = fma(-alpha, v, r);
    pn = fma(dinv, rn, beta * p);
}

template <typename T>
__device__ __forceinline__ T x_update(T x, T r, T p, T dinv, T alpha, T ratio)
{
    return fma(ratio, fma(-dinv, r, p), fma(alpha, p, x));
}

/* Deterministic reduction of NV values over a block into out[0..NV). */
template <typename T, int NV, int WG>
__device__ __forceinline__ void block_reduce(T (&acc)[NV], T *red, T *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        T s = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[wave * NV + c] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        T s = 0;
        for (int w = 0; w < WG / 64; ++w) s += red[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

/* Fixed-order sums of the seven inner products over nparts per-block
 * partial records (8 doubles each, 7 used), then the scalar update of
 * Algorithm 5 into the device state.  Called by one block. */
template <typename T, typename ARGS>
__device__ void finish_iteration(const ARGS &a, int64_t nparts, T *red)
{
    /* fixed-order sums of the 7 inner products over all per-block partials;
     * every thread owns a fixed strided subset, loads issued 4 records at a time */
    T acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = 0;
    for (int64_t b0 = threadIdx.x; b0 < nparts; b0 += 4 * SHARED_WG) {
        T rec[4][7];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t b = b0 + (int64_t)u * SHARED_WG;
#pragma unroll
            for (int c = 0; c < 7; ++c) rec[u][c] = b < nparts ? a.dots[b * 8 + c] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[c] += rec[u][c];
    }
    __shared__ T tot[8];
    block_reduce<T, 7, SHARED_WG>(acc, red, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        CGState *st = a.st;
        const T gam = tot[0], pa = tot[1], rb = tot[2], vc = tot[3], dd = tot[4], ee = tot[5], ff = tot[6];
        const int k = st->k + 1;
        const T prev_ratio = st->beta != 0.0 ? (T)(st->alpha / st->beta) : (T)0;
        const bool bad = !(pa > 0) || !isfinite(pa) || !isfinite(gam) || !isfinite(dd) || !isfinite(vc);
        if (bad) {
            st->flag = FLAG_BREAK;
            st->xa = 0.0;
            st->xratio = (double)prev_ratio;
            st->k = k;
            return;
        }
        const T alpha = dd / pa;
        T rho2 = gam - 2 * alpha * rb + alpha * alpha * vc;
        const T rho = sqrt(rho2 > 0 ? rho2 : (T)0);
        a.hist[k] = (double)rho;
        st->xa = (double)alpha;
        st->xratio = (double)prev_ratio;
        if ((double)rho < st->eps) {
            st->flag = FLAG_CONV;
        } else {
            const T beta = (dd - 2 * alpha * ee + alpha * alpha * ff) / dd;
            if (!(beta != 0) || !isfinite(beta)) {
                st->flag = (beta == 0) ? FLAG_CONV : FLAG_BREAK;
            } else {
                st->ratio = (double)prev_ratio;
                st->alpha = (double)alpha;
                st->beta = (double)beta;
            }
        }
        st->k = k;
    }
}

}  // namespace mfcg
