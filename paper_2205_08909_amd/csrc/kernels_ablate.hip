/*
 * kernels_ablate.hip -- the two comparison solvers the fused iteration is
 * measured against, built from the same operator kernels (the fused tile
 * kernel and the shared-node kernel in their plain mat-vec mode) plus
 * separate streaming vector kernels:
 *
 *  Algorithm 5 split into three passes (the scheme the paper uses on the
 *  GPU, Sec. 6): a "pre" kernel over all entries (r, p and, every other
 *  iteration, x), the mat-vec v = A p, and a "post" kernel with the seven
 *  inner products; the same one-block finish as the fused path.
 *
 *  Basic Jacobi-PCG (Algorithm 1): separate kernels for r^T D^{-1} r, the
 *  search direction, the mat-vec, p^T v and the x/r update with ||r||,
 *  each reduction finished by one block on the device.
 *
 * Both also run with M = I (PREC = false: the diagonal is never read),
 * which makes them Algorithm 4 split into passes and the textbook CG.
 *
 * The vector kernels are grid-stride loops over the internal vector order;
 * every partial sum is reduced in a fixed order, so runs are reproducible.
 */
#include <hip/hip_runtime.h>

#include "cg_common.h"
#include "kernels.h"

namespace mfcg {

constexpr int VEC_WG = 256;
constexpr int VEC_PER_THREAD = 4; /* entries per thread that size the grid */

/* ---------------- Algorithm 5, three passes ---------------- */

template <bool PREC>
__global__ __launch_bounds__(VEC_WG) void alg5_pre_kernel(const IterArgs<double> a, int64_t n)
{
    const CGState *st = a.st;
    if (st->flag != FLAG_RUN) return;
    const double alpha = st->alpha, beta = st->beta, ratio = st->ratio;
    const int kk = st->k + 1;
    const bool xupd = (kk > 1) && (kk & 1);
    const int64_t stride = (int64_t)gridDim.x * VEC_WG;
    for (int64_t i = (int64_t)blockIdx.x * VEC_WG + threadIdx.x; i < n; i += stride) {
        const double r0 = a.r[i], v0 = a.v[i], p0 = a.p[i], dv = PREC ? a.dinv[i] : 1.0;
        double rn, pn;
        pre_update(r0, v0, p0, dv, alpha, beta, rn, pn);
        if (xupd) a.x[i] = x_update(a.x[i], r0, p0, dv, alpha, ratio);
        a.r[i] = rn;
        a.p[i] = pn;
    }
}

template <bool PREC>
__global__ __launch_bounds__(VEC_WG) void alg5_post_kernel(const IterArgs<double> a, int64_t n)
{
    __shared__ double red[8 * (VEC_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    double acc[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = 0;
    const int64_t stride = (int64_t)gridDim.x * VEC_WG;
    for (int64_t i = (int64_t)blockIdx.x * VEC_WG + threadIdx.x; i < n; i += stride) {
        const double r = a.r[i], p = a.p[i], v = a.v[i], dv = PREC ? a.dinv[i] : 1.0;
        const double zr = dv * r, zv = dv * v;
        acc[0] += r * r;
        acc[1] += p * v;
        acc[2] += r * v;
        acc[3] += v * v;
        acc[4] += r * zr;
        acc[5] += r * zv;
        acc[6] += v * zv;
    }
    block_reduce<double, 7, VEC_WG>(acc, red, a.dots + (int64_t)blockIdx.x * 8);
}

__global__ __launch_bounds__(SHARED_WG) void alg5_finish_kernel(const IterArgs<double> a, int64_t nparts)
{
    __shared__ double red[8 * (SHARED_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    finish_iteration<double>(a, nparts, red);
}

/* ---------------- Algorithm 1 (basic PCG) ---------------- */

/* which == 0: sum r_i^2 dinv_i (r_i^2 without preconditioner);  1: sum p_i v_i */
template <int WHICH, bool PREC>
__global__ __launch_bounds__(VEC_WG) void pcg_dot_kernel(const IterArgs<double> a, int64_t n)
{
    __shared__ double red[8 * (VEC_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * VEC_WG;
    for (int64_t i = (int64_t)blockIdx.x * VEC_WG + threadIdx.x; i < n; i += stride) {
        if (WHICH == 0) {
            const double r = a.r[i];
            acc[0] += r * ((PREC ? a.dinv[i] : 1.0) * r);
        } else {
            acc[0] += a.p[i] * a.v[i];
        }
    }
    block_reduce<double, 1, VEC_WG>(acc, red, a.dots + (int64_t)blockIdx.x * 8);
}

/* p = D^{-1} r + beta p */
template <bool PREC>
__global__ __launch_bounds__(VEC_WG) void pcg_p_kernel(const IterArgs<double> a, int64_t n)
{
    if (a.st->flag != FLAG_RUN) return;
    const double beta = a.st->beta;
    const int64_t stride = (int64_t)gridDim.x * VEC_WG;
    for (int64_t i = (int64_t)blockIdx.x * VEC_WG + threadIdx.x; i < n; i += stride)
        a.p[i] = fma(PREC ? a.dinv[i] : 1.0, a.r[i], beta * a.p[i]);
}

/* x += alpha p, r -= alpha v, partial ||r||^2 */
__global__ __launch_bounds__(VEC_WG) void pcg_xr_kernel(const IterArgs<double> a, int64_t n)
{
    __shared__ double red[8 * (VEC_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    const double alpha = a.st->alpha;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * VEC_WG;
    for (int64_t i = (int64_t)blockIdx.x * VEC_WG + threadIdx.x; i < n; i += stride) {
        a.x[i] = fma(alpha, a.p[i], a.x[i]);
        const double r = fma(-alpha, a.v[i], a.r[i]);
        a.r[i] = r;
        acc[0] += r * r;
    }
    block_reduce<double, 1, VEC_WG>(acc, red, a.dots + (int64_t)blockIdx.x * 8);
}

/* one block: fixed-order sum of the first entry of nparts records */
__device__ double sum_parts(const double *dots, int64_t nparts, double *red)
{
    double acc[1] = {0.0};
    for (int64_t b = threadIdx.x; b < nparts; b += SHARED_WG) acc[0] += dots[b * 8];
    __shared__ double tot[8];
    block_reduce<double, 1, SHARED_WG>(acc, red, tot);
    __syncthreads();
    return tot[0];
}

/* STAGE 0: rz_new -> beta (0 in the first iteration);
 * STAGE 1: p^T v -> alpha;
 * STAGE 2: ||r|| -> history, iteration count, convergence test. */
template <int STAGE>
__global__ __launch_bounds__(SHARED_WG) void pcg_finish_kernel(const IterArgs<double> a, int64_t nparts)
{
    __shared__ double red[8 * (SHARED_WG / 64)];
    CGState *st = a.st;
    if (st->flag != FLAG_RUN) return;
    const double s = sum_parts(a.dots, nparts, red);
    if (threadIdx.x != 0) return;
    if (STAGE == 0) {
        if (s == 0.0) {
            st->flag = FLAG_CONV;
        } else if (!(s > 0) || !isfinite(s)) {
            st->flag = FLAG_BREAK;
        } else {
            st->beta = st->k == 0 ? 0.0 : s / st->rz;
            st->rz = s;
        }
    } else if (STAGE == 1) {
        if (!(s > 0) || !isfinite(s)) {
            st->flag = FLAG_BREAK;
            st->k += 1;
        } else {
            st->alpha = st->rz / s;
        }
    } else {
        const int k = st->k + 1;
        const double rho = sqrt(s);
        a.hist[k] = rho;
        st->k = k;
        if (!isfinite(rho)) st->flag = FLAG_BREAK;
        else if (rho < st->eps) st->flag = FLAG_CONV;
    }
}

/* ---------------- launch wrappers ---------------- */

int vec_blocks(int64_t n)
{
    int64_t b = (n + (int64_t)VEC_WG * VEC_PER_THREAD - 1) / ((int64_t)VEC_WG * VEC_PER_THREAD);
    if (b < 1) b = 1;
    if (b > MAX_VEC_BLOCKS) b = MAX_VEC_BLOCKS;
    return (int)b;
}

hipError_t launch_alg5_pre(const IterArgs<double> &a, int64_t n, bool prec, hipStream_t s)
{
    if (prec)
        hipLaunchKernelGGL(alg5_pre_kernel<true>, dim3(vec_blocks(n)), dim3(VEC_WG), 0, s, a, n);
    else
        hipLaunchKernelGGL(alg5_pre_kernel<false>, dim3(vec_blocks(n)), dim3(VEC_WG), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_alg5_post(const IterArgs<double> &a, int64_t n, bool prec, hipStream_t s)
{
    const int nb = vec_blocks(n);
    if (prec)
        hipLaunchKernelGGL(alg5_post_kernel<true>, dim3(nb), dim3(VEC_WG), 0, s, a, n);
    else
        hipLaunchKernelGGL(alg5_post_kernel<false>, dim3(nb), dim3(VEC_WG), 0, s, a, n);
    hipLaunchKernelGGL(alg5_finish_kernel, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    return hipGetLastError();
}

hipError_t launch_pcg_direction(const IterArgs<double> &a, int64_t n, bool prec, hipStream_t s)
{
    const int nb = vec_blocks(n);
    if (prec)
        hipLaunchKernelGGL((pcg_dot_kernel<0, true>), dim3(nb), dim3(VEC_WG), 0, s, a, n);
    else
        hipLaunchKernelGGL((pcg_dot_kernel<0, false>), dim3(nb), dim3(VEC_WG), 0, s, a, n);
    hipLaunchKernelGGL(pcg_finish_kernel<0>, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    if (prec)
        hipLaunchKernelGGL(pcg_p_kernel<true>, dim3(nb), dim3(VEC_WG), 0, s, a, n);
    else
        hipLaunchKernelGGL(pcg_p_kernel<false>, dim3(nb), dim3(VEC_WG), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_pcg_update(const IterArgs<double> &a, int64_t n, hipStream_t s)
{
    const int nb = vec_blocks(n);
    hipLaunchKernelGGL((pcg_dot_kernel<1, true>), dim3(nb), dim3(VEC_WG), 0, s, a, n);
    hipLaunchKernelGGL(pcg_finish_kernel<1>, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    hipLaunchKernelGGL(pcg_xr_kernel, dim3(nb), dim3(VEC_WG), 0, s, a, n);
    hipLaunchKernelGGL(pcg_finish_kernel<2>, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    return hipGetLastError();
}

}  // namespace mfcg
