/*
 * nn_kernels.hip -- kernels of the learned warm start's small 3D
 * convolutional network, written for gfx950: BF16 storage of activations
 * and weights, FP32 accumulation, NCDHW layout (W fastest, which is the
 * x-fastest lexicographic node order of the solver's vectors).
 *
 * The 32 -> 32 channel layers of stride 1 (forward and data gradient) run
 * as implicit GEMMs on the BF16 matrix cores (conv_mfma_kernel).  The other
 * shapes (3 -> 32 channels at stride 4, the 32 -> 1 transposed layer, the
 * weight gradients) are direct convolutions that keep each thread's output
 * channels in registers and the layer's weights in LDS (as FP32, read as
 * broadcasts).
 *
 *   conv_fwd_kernel        y = act(conv(x, w) + b)
 *   conv_bwd_data_kernel   dx = conv(., w)^T g (+ b per input channel: the
 *                          forward map of a transposed convolution)
 *   conv_bwd_weight_kernel per-chunk partial sums of dw, reduced in a fixed
 *                          order by conv_wsum_kernel; conv_bsum_kernel: db
 *   act_bwd_kernel, mse_kernel (+ mse_sum_kernel), adam_kernel,
 *   convert_kernel, feature kernels.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_kernels.h"

namespace mfnn {

constexpr int NN_WG = 256;

/* BF16 <-> FP32: BF16 is the upper half of the FP32 bit pattern; rounding
 * to nearest, ties to even, NaN kept quiet. */
__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename T>
__device__ __forceinline__ float load_f(const T *p, int64_t i);
template <>
__device__ __forceinline__ float load_f<uint16_t>(const uint16_t *p, int64_t i) { return bf16_to_f32(p[i]); }
template <>
__device__ __forceinline__ float load_f<float>(const float *p, int64_t i) { return p[i]; }

template <typename T>
__device__ __forceinline__ void store_f(T *p, int64_t i, float v);
template <>
__device__ __forceinline__ void store_f<uint16_t>(uint16_t *p, int64_t i, float v) { p[i] = f32_to_bf16(v); }
template <>
__device__ __forceinline__ void store_f<float>(float *p, int64_t i, float v) { p[i] = v; }

__device__ __forceinline__ float leaky(float z) { return z > 0.f ? z : LEAKY_SLOPE * z; }

/* ---------------- forward ---------------- */

/* One thread: one output point, COT consecutive output channels
 * (blockIdx.y selects the group).  LDS: wl[(ci*T + t)*COT + c] = w[co0+c][ci][t]. */
template <typename TI, typename TO, int COT>
__global__ __launch_bounds__(NN_WG) void conv_fwd_kernel(const ConvGeom g, const TI *__restrict__ x,
                                                         const uint16_t *__restrict__ w,
                                                         const float *__restrict__ bias, int act,
                                                         TO *__restrict__ y)
{
    extern __shared__ float wl[];
    const int T = g.k[0] * g.k[1] * g.k[2];
    const int co0 = blockIdx.y * COT;
    const int nw = g.ci * T * COT;
    for (int e = threadIdx.x; e < nw; e += NN_WG) {
        const int c = e % COT, rest = e / COT; /* rest = ci*T + t */
        wl[e] = bf16_to_f32(w[(int64_t)(co0 + c) * g.ci * T + rest]);
    }
    __syncthreads();
    const int64_t ovox = (int64_t)g.out[0] * g.out[1] * g.out[2];
    const int64_t v = (int64_t)blockIdx.x * NN_WG + threadIdx.x;
    if (v >= (int64_t)g.n * ovox) return;
    const int n = (int)(v / ovox);
    int64_t r = v - (int64_t)n * ovox;
    const int ox = (int)(r % g.out[2]);
    r /= g.out[2];
    const int oy = (int)(r % g.out[1]);
    const int oz = (int)(r / g.out[1]);
    const int64_t ivox = (int64_t)g.in[0] * g.in[1] * g.in[2];
    float acc[COT];
#pragma unroll
    for (int c = 0; c < COT; ++c) acc[c] = 0.f;
    for (int ci = 0; ci < g.ci; ++ci) {
        const TI *xc = x + ((int64_t)n * g.ci + ci) * ivox;
        for (int tz = 0; tz < g.k[0]; ++tz) {
            const int iz = oz * g.s[0] - g.p[0] + tz * g.d[0];
            if (iz < 0 || iz >= g.in[0]) continue;
            for (int ty = 0; ty < g.k[1]; ++ty) {
                const int iy = oy * g.s[1] - g.p[1] + ty * g.d[1];
                if (iy < 0 || iy >= g.in[1]) continue;
                const int64_t rowb = ((int64_t)iz * g.in[1] + iy) * g.in[2];
                const int tb = (tz * g.k[1] + ty) * g.k[2];
                for (int tx = 0; tx < g.k[2]; ++tx) {
                    const int ix = ox * g.s[2] - g.p[2] + tx * g.d[2];
                    if (ix < 0 || ix >= g.in[2]) continue;
                    const float xv = load_f(xc, rowb + ix);
                    const float *wp = wl + ((int64_t)ci * T + tb + tx) * COT;
#pragma unroll
                    for (int c = 0; c < COT; ++c) acc[c] = fmaf(wp[c], xv, acc[c]);
                }
            }
        }
    }
    const int64_t obase = ((int64_t)n * g.co + co0) * ovox + (v - (int64_t)n * ovox);
#pragma unroll
    for (int c = 0; c < COT; ++c) {
        float z = acc[c] + (bias ? bias[co0 + c] : 0.f);
        if (act == ACT_LEAKY) z = leaky(z);
        store_f(y, obase + (int64_t)c * ovox, z);
    }
}

/* ---------------- backward data / transposed forward ---------------- */

/* One thread: one input point, CIT consecutive input channels.
 * LDS: wl[(co*T + t)*CIT + c] = w[co][ci0+c][t]. */
template <typename TG, typename TO, int CIT>
__global__ __launch_bounds__(NN_WG) void conv_bwd_data_kernel(const ConvGeom g, const TG *__restrict__ gr,
                                                              const uint16_t *__restrict__ w,
                                                              const float *__restrict__ bias_in,
                                                              TO *__restrict__ dx)
{
    extern __shared__ float wl[];
    const int T = g.k[0] * g.k[1] * g.k[2];
    const int ci0 = blockIdx.y * CIT;
    const int nw = g.co * T * CIT;
    for (int e = threadIdx.x; e < nw; e += NN_WG) {
        const int c = e % CIT, rest = e / CIT; /* rest = co*T + t */
        const int co = rest / T, t = rest - co * T;
        wl[e] = bf16_to_f32(w[((int64_t)co * g.ci + ci0 + c) * T + t]);
    }
    __syncthreads();
    const int64_t ivox = (int64_t)g.in[0] * g.in[1] * g.in[2];
    const int64_t v = (int64_t)blockIdx.x * NN_WG + threadIdx.x;
    if (v >= (int64_t)g.n * ivox) return;
    const int n = (int)(v / ivox);
    int64_t r = v - (int64_t)n * ivox;
    const int ix = (int)(r % g.in[2]);
    r /= g.in[2];
    const int iy = (int)(r % g.in[1]);
    const int iz = (int)(r / g.in[1]);
    const int64_t ovox = (int64_t)g.out[0] * g.out[1] * g.out[2];
    float acc[CIT];
#pragma unroll
    for (int c = 0; c < CIT; ++c) acc[c] = 0.f;
    for (int tz = 0; tz < g.k[0]; ++tz) {
        const int nz = iz + g.p[0] - tz * g.d[0];
        if (nz < 0 || nz % g.s[0]) continue;
        const int oz = nz / g.s[0];
        if (oz >= g.out[0]) continue;
        for (int ty = 0; ty < g.k[1]; ++ty) {
            const int ny = iy + g.p[1] - ty * g.d[1];
            if (ny < 0 || ny % g.s[1]) continue;
            const int oy = ny / g.s[1];
            if (oy >= g.out[1]) continue;
            for (int tx = 0; tx < g.k[2]; ++tx) {
                const int nx = ix + g.p[2] - tx * g.d[2];
                if (nx < 0 || nx % g.s[2]) continue;
                const int ox = nx / g.s[2];
                if (ox >= g.out[2]) continue;
                const int t = (tz * g.k[1] + ty) * g.k[2] + tx;
                const int64_t ob = ((int64_t)oz * g.out[1] + oy) * g.out[2] + ox;
                for (int co = 0; co < g.co; ++co) {
                    const float gv = load_f(gr, ((int64_t)n * g.co + co) * ovox + ob);
                    const float *wp = wl + ((int64_t)co * T + t) * CIT;
#pragma unroll
                    for (int c = 0; c < CIT; ++c) acc[c] = fmaf(wp[c], gv, acc[c]);
                }
            }
        }
    }
    const int64_t ib = ((int64_t)n * g.ci + ci0) * ivox + (v - (int64_t)n * ivox);
#pragma unroll
    for (int c = 0; c < CIT; ++c) store_f(dx, ib + (int64_t)c * ivox, acc[c] + (bias_in ? bias_in[ci0 + c] : 0.f));
}

/* ---------------- backward weight ---------------- */

template <int NV>
__device__ __forceinline__ void block_sum(float (&acc)[NV], float *red, float *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        float s = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[wave * NV + c] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        float s = 0.f;
        for (int w = 0; w < NN_WG / 64; ++w) s += red[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

/* blockIdx.x = ci*T + t, blockIdx.y = chunk of the (n, o) points,
 * blockIdx.z = group of WCO output channels.
 * part[((chunk*co + co)*ci + ci)*T + t] = sum over the chunk of g * x. */
template <typename TX, typename TG, int WCO>
__global__ __launch_bounds__(NN_WG) void conv_bwd_weight_kernel(const ConvGeom g, const TX *__restrict__ x,
                                                                const TG *__restrict__ gr, float *__restrict__ part)
{
    __shared__ float red[WCO * (NN_WG / 64)];
    const int T = g.k[0] * g.k[1] * g.k[2];
    const int ci = blockIdx.x / T, t = blockIdx.x - ci * T;
    const int tz = t / (g.k[1] * g.k[2]), ty = (t / g.k[2]) % g.k[1], tx = t % g.k[2];
    const int co0 = blockIdx.z * WCO;
    const int64_t ovox = (int64_t)g.out[0] * g.out[1] * g.out[2];
    const int64_t ivox = (int64_t)g.in[0] * g.in[1] * g.in[2];
    const int64_t V = (int64_t)g.n * ovox;
    const int64_t c0 = V * blockIdx.y / gridDim.y, c1 = V * (blockIdx.y + 1) / gridDim.y;
    float acc[WCO];
#pragma unroll
    for (int c = 0; c < WCO; ++c) acc[c] = 0.f;
    for (int64_t v = c0 + threadIdx.x; v < c1; v += NN_WG) {
        const int n = (int)(v / ovox);
        const int64_t o = v - (int64_t)n * ovox;
        int64_t r = o;
        const int ox = (int)(r % g.out[2]);
        r /= g.out[2];
        const int oy = (int)(r % g.out[1]);
        const int oz = (int)(r / g.out[1]);
        const int iz = oz * g.s[0] - g.p[0] + tz * g.d[0];
        const int iy = oy * g.s[1] - g.p[1] + ty * g.d[1];
        const int ix = ox * g.s[2] - g.p[2] + tx * g.d[2];
        if (iz < 0 || iz >= g.in[0] || iy < 0 || iy >= g.in[1] || ix < 0 || ix >= g.in[2]) continue;
        const float xv = load_f(x, ((int64_t)n * g.ci + ci) * ivox + ((int64_t)iz * g.in[1] + iy) * g.in[2] + ix);
        const int64_t gb = ((int64_t)n * g.co + co0) * ovox + o;
#pragma unroll
        for (int c = 0; c < WCO; ++c) acc[c] = fmaf(load_f(gr, gb + (int64_t)c * ovox), xv, acc[c]);
    }
    __shared__ float tot[WCO];
    block_sum<WCO>(acc, red, tot);
    if (threadIdx.x < WCO)
        part[(((int64_t)blockIdx.y * g.co + co0 + threadIdx.x) * g.ci + ci) * T + t] = tot[threadIdx.x];
}

/* dw[e] = sum over chunks (fixed order) of part[chunk*nw + e] */
__global__ __launch_bounds__(NN_WG) void conv_wsum_kernel(int64_t nw, int nchunks, const float *__restrict__ part,
                                                          float *__restrict__ dw)
{
    const int64_t e = (int64_t)blockIdx.x * NN_WG + threadIdx.x;
    if (e >= nw) return;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * nw + e];
    dw[e] = s;
}

/* db[co] = sum over (n, o) of g; one block per output channel */
template <typename TG>
__global__ __launch_bounds__(NN_WG) void conv_bsum_kernel(const ConvGeom g, const TG *__restrict__ gr,
                                                          float *__restrict__ db)
{
    __shared__ float red[NN_WG / 64];
    const int co = blockIdx.x;
    const int64_t ovox = (int64_t)g.out[0] * g.out[1] * g.out[2];
    float acc[1] = {0.f};
    for (int n = 0; n < g.n; ++n) {
        const TG *gp = gr + ((int64_t)n * g.co + co) * ovox;
        for (int64_t o = threadIdx.x; o < ovox; o += NN_WG) acc[0] += load_f(gp, o);
    }
    __shared__ float tot[1];
    block_sum<1>(acc, red, tot);
    if (threadIdx.x == 0) db[co] = tot[0];
}

/* The same sum spread over nb blocks per channel: part[co * nb + b] = the
 * sum of slice b of channel co's (n, o) points (fixed slices, fixed order
 * inside a block); csum_finish_kernel adds a channel's nb partials in
 * order.  A single block per channel reads at the bandwidth of one compute
 * unit, which takes milliseconds on a fine grid. */
template <typename TG>
__global__ __launch_bounds__(NN_WG) void csum_part_kernel(const ConvGeom g, const TG *__restrict__ gr, int nb,
                                                          float *__restrict__ part)
{
    __shared__ float red[NN_WG / 64];
    const int co = blockIdx.y, b = blockIdx.x;
    const int64_t ovox = (int64_t)g.out[0] * g.out[1] * g.out[2];
    const int64_t V = (int64_t)g.n * ovox;
    const int64_t v0 = V * b / nb, v1 = V * (b + 1) / nb;
    float acc[1] = {0.f};
    for (int64_t v = v0 + threadIdx.x; v < v1; v += NN_WG) {
        const int n = (int)(v / ovox);
        acc[0] += load_f(gr, ((int64_t)n * g.co + co) * ovox + (v - (int64_t)n * ovox));
    }
    __shared__ float tot[1];
    block_sum<1>(acc, red, tot);
    if (threadIdx.x == 0) part[(int64_t)co * nb + b] = tot[0];
}

__global__ void csum_finish_kernel(int c, int nb, const float *__restrict__ part, float *__restrict__ out)
{
    const int co = blockIdx.x * blockDim.x + threadIdx.x;
    if (co >= c) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)co * nb + b];
    out[co] = s;
}

/* out[co] = sum of g over (n, o) per channel; with work (at least co
 * floats per block), nb blocks per channel and a fixed-order finish */
template <typename TG>
static hipError_t channel_sum_t(const ConvGeom &g, const void *gr, float *out, float *work, int64_t work_floats,
                                hipStream_t s)
{
    const int64_t V = (int64_t)g.n * g.out[0] * g.out[1] * g.out[2];
    int64_t nb = work ? work_floats / g.co : 0;
    if (nb > CSUM_MAX_BLOCKS) nb = CSUM_MAX_BLOCKS;
    if (nb > (V + NN_WG - 1) / NN_WG) nb = (V + NN_WG - 1) / NN_WG;
    if (nb < 2) {
        hipLaunchKernelGGL((conv_bsum_kernel<TG>), dim3(g.co), dim3(NN_WG), 0, s, g, (const TG *)gr, out);
    } else {
        hipLaunchKernelGGL((csum_part_kernel<TG>), dim3((unsigned)nb, g.co), dim3(NN_WG), 0, s, g, (const TG *)gr,
                           (int)nb, work);
        hipLaunchKernelGGL(csum_finish_kernel, dim3((g.co + 63) / 64), dim3(64), 0, s, g.co, (int)nb,
                           (const float *)work, out);
    }
    return hipGetLastError();
}

/* ---------------- elementwise ---------------- */

template <typename TY>
__global__ __launch_bounds__(NN_WG) void act_bwd_kernel(int64_t n, const float *__restrict__ dy,
                                                        const TY *__restrict__ y, float *__restrict__ dz)
{
    for (int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NN_WG)
        dz[i] = load_f(y, i) > 0.f ? dy[i] : LEAKY_SLOPE * dy[i];
}

/* grad = 2 (pred - target) / n; part[b] = block partial of (pred - target)^2 (FP64) */
__global__ __launch_bounds__(NN_WG) void mse_kernel(int64_t n, const float *__restrict__ pred,
                                                    const float *__restrict__ target, float *__restrict__ grad,
                                                    double *__restrict__ part)
{
    __shared__ double red[NN_WG / 64];
    double acc = 0.0;
    const float sc = 2.0f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NN_WG) {
        const float r = pred[i] - target[i];
        grad[i] = sc * r;
        acc += (double)r * r;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NN_WG / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(64) void mse_sum_kernel(int nb, int64_t n, const double *__restrict__ part,
                                                     double *__restrict__ loss)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    *loss = s / (double)n;
}

__global__ __launch_bounds__(NN_WG) void adam_kernel(int64_t n, float *__restrict__ th, uint16_t *__restrict__ thb,
                                                     const float *__restrict__ gr, float *__restrict__ m,
                                                     float *__restrict__ v, float lr, float b1, float b2, float eps,
                                                     float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NN_WG) {
        const float g = gr[i];
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        const float t = th[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        th[i] = t;
        if (thb) thb[i] = f32_to_bf16(t);
    }
}

/* dtype conversions: 0 bf16, 1 f32, 2 f64 */
__global__ __launch_bounds__(NN_WG) void convert_kernel(int64_t n, const void *__restrict__ in, int tin,
                                                        void *__restrict__ out, int tout)
{
    for (int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NN_WG) {
        double v;
        if (tin == DT_BF16) v = bf16_to_f32(((const uint16_t *)in)[i]);
        else if (tin == DT_F32) v = ((const float *)in)[i];
        else v = ((const double *)in)[i];
        if (tout == DT_BF16) ((uint16_t *)out)[i] = f32_to_bf16((float)v);
        else if (tout == DT_F32) ((float *)out)[i] = (float)v;
        else ((double *)out)[i] = v;
    }
}

/* ---------------- input features ---------------- */

/* part[2b], part[2b+1]: block partials of sum b^2 and sum (b/diag)^2 */
__global__ __launch_bounds__(NN_WG) void feat_norm_kernel(int64_t n, const double *__restrict__ b,
                                                          const double *__restrict__ diag, double *__restrict__ part)
{
    __shared__ double red[2 * (NN_WG / 64)];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NN_WG) {
        const double v = b[i], q = v / diag[i];
        a0 += v * v;
        a1 += q * q;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off, 64);
        a1 += __shfl_xor(a1, off, 64);
    }
    if (lane == 0) {
        red[2 * wave] = a0;
        red[2 * wave + 1] = a1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int w = 0; w < NN_WG / 64; ++w) s += red[2 * w + threadIdx.x];
        part[2 * blockIdx.x + threadIdx.x] = s;
    }
}

/* out[0][node] = mean of log a over the cells touching the node;
 * out[1][node] = b / rms(b); out[2][node] = (b / diag) / rms(b / diag). */
__global__ __launch_bounds__(NN_WG) void feat_kernel(FeatGeom f, const double *__restrict__ logc,
                                                     const double *__restrict__ b, const double *__restrict__ diag,
                                                     const double *__restrict__ part, int nb, uint16_t *__restrict__ out)
{
    __shared__ double sc[2];
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int q = 0; q < nb; ++q) s += part[2 * q + threadIdx.x];
        const double rms = sqrt(s / (double)f.n);
        sc[threadIdx.x] = rms > 0.0 ? 1.0 / rms : 0.0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x;
    if (i >= f.n) return;
    const int L0 = f.cells[0] * f.k + 1, L1 = f.cells[1] * f.k + 1;
    const int nx = (int)(i % L0), ny = (int)((i / L0) % L1), nz = (int)(i / ((int64_t)L0 * L1));
    int lo[3], hi[3];
    const int nd[3] = {nx, ny, nz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int c = nd[d] / f.k;
        if (nd[d] % f.k == 0) {
            lo[d] = c > 0 ? c - 1 : 0;
            hi[d] = c < f.cells[d] ? c : f.cells[d] - 1;
        } else {
            lo[d] = hi[d] = c;
        }
    }
    double s = 0.0;
    int cnt = 0;
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
        for (int cy = lo[1]; cy <= hi[1]; ++cy)
            for (int cx = lo[0]; cx <= hi[0]; ++cx) {
                s += logc[cx + (int64_t)f.cells[0] * (cy + (int64_t)f.cells[1] * cz)];
                ++cnt;
            }
    out[i] = f32_to_bf16((float)(s / cnt));
    out[f.n + i] = f32_to_bf16((float)(b[i] * sc[0]));
    out[2 * f.n + i] = f32_to_bf16((float)(b[i] / diag[i] * sc[1]));
}

/* out = in / rms(in) (FP64 in, FP32 out); part: FEAT_NORM_BLOCKS partials */
__global__ __launch_bounds__(NN_WG) void sumsq64_kernel(int64_t n, const double *__restrict__ in,
                                                        double *__restrict__ part)
{
    __shared__ double red[NN_WG / 64];
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NN_WG) a += in[i] * in[i];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) red[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NN_WG / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(NN_WG) void normalize_kernel(int64_t n, const double *__restrict__ in,
                                                          const double *__restrict__ part, int nb,
                                                          float *__restrict__ out)
{
    __shared__ double sc;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < nb; ++q) s += part[q];
        const double rms = sqrt(s / (double)n);
        sc = rms > 0.0 ? 1.0 / rms : 0.0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NN_WG + threadIdx.x;
    if (i < n) out[i] = (float)(in[i] * sc);
}

/* ---------------- launch wrappers ---------------- */

static unsigned grid_for(int64_t n)
{
    int64_t b = (n + NN_WG - 1) / NN_WG;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

/* ---------------- matrix-core path: 32 -> 32 channels, stride 1 ---------------- */

/* The dense layers of the network (32 input and 32 output channels, a
 * cubic kernel of K^3 taps with dilation d, stride 1) as an implicit GEMM
 * on the BF16 matrix cores: per tap, out[oc][point] += W[oc][ic] x[ic][point
 * shifted by the tap], a 32 x 32 x 8 product (v_mfma_f32_32x32x8_bf16) per
 * block of 8 input channels, FP32 accumulation.  A workgroup of 4 waves
 * owns 128 consecutive output points of one z-plane (a wave per 32-point
 * block, the matrix N dimension); for each z-tap it stages the K^2 taps'
 * weights and the input rows the block needs (all 32 channels, channel
 * fastest, zero outside the input) in LDS, then every wave runs the K^2 x 4
 * products of that plane.  flip = 1 reads the weights as w[ic][oc][T-1-t]:
 * the data gradient of a stride-1 convolution with symmetric padding is
 * this convolution of the output gradient with the flipped, transposed
 * kernel. */
typedef short mf_v4s __attribute__((ext_vector_type(4)));
typedef float mf_v16f __attribute__((ext_vector_type(16)));
constexpr int MF_C = 32, MF_WG = 256, MF_PTS = 128;

struct MfGeom {
    int32_t n;
    int32_t in[3], out[3];
    int32_t K, d, p;
    int32_t flip;
    int32_t SW, RMAX; /* slab columns, slab rows allocated */
};

template <typename TO>
__global__ __launch_bounds__(MF_WG) void conv_mfma_kernel(const MfGeom g, const uint16_t *__restrict__ x,
                                                          const uint16_t *__restrict__ w,
                                                          const float *__restrict__ bias, int act,
                                                          TO *__restrict__ y)
{
    extern __shared__ uint16_t mf_lds[];
    const int K = g.K, K2 = K * K, T = K2 * K;
    uint16_t *wl = mf_lds;                /* K^2 taps x 32 oc x 32 ic */
    uint16_t *xs = wl + K2 * MF_C * MF_C; /* RMAX x SW points x 32 ic */
    const int64_t plane = (int64_t)g.out[1] * g.out[2];
    const int64_t pblocks = (plane + MF_PTS - 1) / MF_PTS;
    const int64_t bid = blockIdx.x;
    const int64_t pb = bid % pblocks, rest = bid / pblocks;
    const int oz = (int)(rest % g.out[0]), n = (int)(rest / g.out[0]);
    const int64_t q0 = pb * MF_PTS;
    const int64_t qlast = (q0 + MF_PTS < plane ? q0 + MF_PTS : plane) - 1;
    const int oy0 = (int)(q0 / g.out[2]), oy1 = (int)(qlast / g.out[2]);
    const int SR = oy1 - oy0 + 1 + (K - 1) * g.d; /* <= RMAX by the launch's choice of RMAX */
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q = q0 + wave * 32 + (lane & 31);
    const bool qv = q < plane;
    const int64_t qc = qv ? q : q0;
    const int oy = (int)(qc / g.out[2]), ox = (int)(qc - (int64_t)oy * g.out[2]);
    const int sbase = (oy - oy0) * g.SW + ox;
    const int khalf = (lane >> 5) * 4;
    const int64_t ivox = (int64_t)g.in[0] * g.in[1] * g.in[2];
    mf_v16f acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    for (int tz = 0; tz < K; ++tz) {
        const int iz = oz - g.p + tz * g.d;
        if (iz < 0 || iz >= g.in[0]) continue; /* the same for the whole workgroup */
        __syncthreads();                       /* the previous plane's products are done */
        for (int e = threadIdx.x; e < K2 * MF_C * MF_C; e += MF_WG) {
            const int ic = e & 31, oc = (e >> 5) & 31, tyx = e >> 10;
            const int t = tz * K2 + tyx;
            wl[e] = g.flip ? w[((int64_t)ic * MF_C + oc) * T + (T - 1 - t)] : w[((int64_t)oc * MF_C + ic) * T + t];
        }
        const int nel = SR * g.SW * MF_C;
        for (int e = threadIdx.x; e < nel; e += MF_WG) {
            const int col = e % g.SW, r2 = e / g.SW;
            const int row = r2 % SR, ic = r2 / SR;
            const int iy = oy0 - g.p + row, ix = col - g.p;
            uint16_t v = 0;
            if (iy >= 0 && iy < g.in[1] && ix >= 0 && ix < g.in[2])
                v = x[((int64_t)n * MF_C + ic) * ivox + ((int64_t)iz * g.in[1] + iy) * g.in[2] + ix];
            xs[(row * g.SW + col) * MF_C + ic] = v;
        }
        __syncthreads();
        for (int ty = 0; ty < K; ++ty)
            for (int tx = 0; tx < K; ++tx) {
                const uint16_t *wb = wl + ((ty * K + tx) * MF_C + (lane & 31)) * MF_C + khalf;
                const uint16_t *xb = xs + (sbase + ty * g.d * g.SW + tx * g.d) * MF_C + khalf;
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    const mf_v4s a = *(const mf_v4s *)(wb + kb * 8);
                    const mf_v4s b = *(const mf_v4s *)(xb + kb * 8);
                    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
                }
            }
    }
    if (!qv) return;
    const int64_t ovox = (int64_t)g.out[0] * plane;
    const int64_t ob = (int64_t)n * MF_C * ovox + (int64_t)oz * plane + q;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int oc = 8 * (v >> 2) + khalf + (v & 3);
        float z = acc[v] + (bias ? bias[oc] : 0.f);
        if (act == ACT_LEAKY) z = leaky(z);
        store_f(y, ob + (int64_t)oc * ovox, z);
    }
}

/* Weight gradient of the same layers on the matrix cores: per tap t,
 * dw[oc][ic][t] = sum over points of g[oc][point] x[ic][point shifted by
 * t], a 32 x 32 x 8 product per 8 points.  A workgroup of 8 waves walks a
 * contiguous range of (sample, z-plane, 128-point block) items; wave w
 * owns the taps t = w, w + 8, ... and keeps their 32 x 32 sums in
 * registers for the whole range.  Per item the output gradient block is
 * staged in LDS as [oc][point] (4 consecutive points per lane in one read)
 * and, per z-tap, the input rows as for the forward map.  Each workgroup
 * writes its partial sums as one chunk; the chunks are added in a fixed
 * order afterwards. */
constexpr int MFW_WAVES = 8, MFW_WG = 64 * MFW_WAVES, MFW_CHUNKS = 32;

template <int K>
__global__ __launch_bounds__(MFW_WG) void conv_wgrad_mfma_kernel(const MfGeom g, const uint16_t *__restrict__ x,
                                                                 const uint16_t *__restrict__ gr,
                                                                 float *__restrict__ part, int nchunks)
{
    extern __shared__ uint16_t mf_lds[];
    constexpr int K2 = K * K, T = K2 * K;
    uint16_t *gs = mf_lds;               /* 32 oc x MF_PTS points */
    uint16_t *xs = gs + MF_C * MF_PTS;   /* RMAX x SW points x 32 ic */
    int *sp0 = (int *)(xs + g.RMAX * g.SW * MF_C); /* slab offset of each point of the block */
    const int64_t plane = (int64_t)g.out[1] * g.out[2];
    const int64_t pblocks = (plane + MF_PTS - 1) / MF_PTS;
    const int64_t nitems = pblocks * g.out[0] * g.n;
    const int64_t it0 = nitems * blockIdx.x / nchunks, it1 = nitems * (blockIdx.x + 1) / nchunks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int khalf = (lane >> 5) * 4, col = lane & 31;
    const int64_t ivox = (int64_t)g.in[0] * g.in[1] * g.in[2];
    const int64_t ovox = (int64_t)g.out[0] * plane;
    constexpr int NT = (T + MFW_WAVES - 1) / MFW_WAVES; /* taps per wave */
    mf_v16f acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[j][v] = 0.f;
    for (int64_t item = it0; item < it1; ++item) {
        const int64_t pb = item % pblocks, rest = item / pblocks;
        const int oz = (int)(rest % g.out[0]), n = (int)(rest / g.out[0]);
        const int64_t q0 = pb * MF_PTS;
        const int64_t qlast = (q0 + MF_PTS < plane ? q0 + MF_PTS : plane) - 1;
        const int oy0 = (int)(q0 / g.out[2]), oy1 = (int)(qlast / g.out[2]);
        const int SR = oy1 - oy0 + 1 + (K - 1) * g.d;
        __syncthreads(); /* the previous item's products are done */
        for (int e = threadIdx.x; e < MF_C * MF_PTS; e += MFW_WG) {
            const int oc = e / MF_PTS, i = e - oc * MF_PTS;
            const int64_t q = q0 + i;
            gs[e] = q < plane ? gr[((int64_t)n * MF_C + oc) * ovox + (int64_t)oz * plane + q] : (uint16_t)0;
        }
        for (int i = threadIdx.x; i < MF_PTS; i += MFW_WG) {
            const int64_t q = q0 + i < plane ? q0 + i : q0; /* points past the plane: g = 0, any valid slab point */
            const int qy = (int)(q / g.out[2]), qx = (int)(q - (int64_t)qy * g.out[2]);
            sp0[i] = (qy - oy0) * g.SW + qx;
        }
        for (int tz = 0; tz < K; ++tz) {
            const int iz = oz - g.p + tz * g.d;
            if (iz < 0 || iz >= g.in[0]) continue; /* the same for the whole workgroup */
            __syncthreads();                       /* the previous plane's products are done */
            const int nel = SR * g.SW * MF_C;
            for (int e = threadIdx.x; e < nel; e += MFW_WG) {
                const int c2 = e % g.SW, r2 = e / g.SW;
                const int row = r2 % SR, ic = r2 / SR;
                const int iy = oy0 - g.p + row, ix = c2 - g.p;
                uint16_t v = 0;
                if (iy >= 0 && iy < g.in[1] && ix >= 0 && ix < g.in[2])
                    v = x[((int64_t)n * MF_C + ic) * ivox + ((int64_t)iz * g.in[1] + iy) * g.in[2] + ix];
                xs[(row * g.SW + c2) * MF_C + ic] = v;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int t = wave + MFW_WAVES * j;
                if (t >= T || t / K2 != tz) continue;
                const int tyx = t - tz * K2, ty = tyx / K, tx = tyx - ty * K;
                const int shift = ty * g.d * g.SW + tx * g.d;
                for (int s8 = 0; s8 < MF_PTS; s8 += 8) {
                    const mf_v4s a = *(const mf_v4s *)(gs + col * MF_PTS + s8 + khalf);
                    mf_v4s b;
#pragma unroll
                    for (int u = 0; u < 4; ++u) b[u] = (short)xs[(sp0[s8 + khalf + u] + shift) * MF_C + col];
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = wave + MFW_WAVES * j;
        if (t >= T) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int oc = 8 * (v >> 2) + khalf + (v & 3);
            part[(((int64_t)blockIdx.x * MF_C + oc) * MF_C + col) * T + t] = acc[j][v];
        }
    }
}

/* The matrix-core geometry of a stride-1, 32 -> 32 channel layer with a
 * cubic kernel, or false when the layer has another shape or its LDS
 * footprint exceeds the budget.  flip: the data-gradient form (needs the
 * symmetric padding 2p = (K-1)d; the gradient has the output's size). */
static bool mfma_geom(const ConvGeom &g, bool flip, MfGeom &m, size_t &lds)
{
    if (g.ci != MF_C || g.co != MF_C) return false;
    for (int i = 0; i < 3; ++i)
        if (g.s[i] != 1 || g.k[i] != g.k[0] || g.d[i] != g.d[0] || g.p[i] != g.p[0]) return false;
    const int K = g.k[0], d = g.d[0], p = g.p[0];
    if (K < 1 || K > 5 || (flip && 2 * p != (K - 1) * d)) return false;
    m = MfGeom{};
    m.n = g.n;
    for (int i = 0; i < 3; ++i) {
        m.in[i] = flip ? g.out[i] : g.in[i];
        m.out[i] = flip ? g.in[i] : g.out[i];
    }
    m.K = K;
    m.d = d;
    m.p = p;
    m.flip = flip ? 1 : 0;
    m.SW = m.out[2] + (K - 1) * d;
    /* rows a block of MF_PTS consecutive points can touch, plus the taps' reach */
    m.RMAX = (MF_PTS - 1) / m.out[2] + 2;
    if (m.RMAX > m.out[1]) m.RMAX = m.out[1];
    m.RMAX += (K - 1) * d;
    lds = ((size_t)K * K * MF_C * MF_C + (size_t)m.RMAX * m.SW * MF_C) * sizeof(uint16_t);
    return lds <= MAX_LDS_BYTES && m.out[0] > 0 && m.out[1] > 0 && m.out[2] > 0;
}

bool mfma_applies(const ConvGeom &g, bool flip)
{
    MfGeom m;
    size_t lds = 0;
    return mfma_geom(g, flip, m, lds);
}

template <typename TO>
static hipError_t mfma_t(const MfGeom &m, size_t lds, const void *x, const uint16_t *w, const float *bias, int act,
                         void *y, hipStream_t s)
{
    const int64_t plane = (int64_t)m.out[1] * m.out[2];
    const int64_t nb = (plane + MF_PTS - 1) / MF_PTS * m.out[0] * m.n;
    hipLaunchKernelGGL((conv_mfma_kernel<TO>), dim3((unsigned)nb), dim3(MF_WG), lds, s, m, (const uint16_t *)x, w,
                       bias, act, (TO *)y);
    return hipGetLastError();
}

template <typename TI, typename TO>
static hipError_t fwd_t(const ConvGeom &g, const void *x, const uint16_t *w, const float *bias, int act, void *y,
                        hipStream_t s)
{
    const int T = g.k[0] * g.k[1] * g.k[2];
    const int64_t tot = (int64_t)g.n * g.out[0] * g.out[1] * g.out[2];
    const unsigned gx = (unsigned)((tot + NN_WG - 1) / NN_WG);
    if (g.co % 8 == 0) {
        hipLaunchKernelGGL((conv_fwd_kernel<TI, TO, 8>), dim3(gx, g.co / 8), dim3(NN_WG),
                           (size_t)g.ci * T * 8 * sizeof(float), s, g, (const TI *)x, w, bias, act, (TO *)y);
    } else {
        hipLaunchKernelGGL((conv_fwd_kernel<TI, TO, 1>), dim3(gx, g.co), dim3(NN_WG), (size_t)g.ci * T * sizeof(float),
                           s, g, (const TI *)x, w, bias, act, (TO *)y);
    }
    return hipGetLastError();
}

hipError_t launch_conv_fwd(const ConvGeom &g, const void *x, int tx, const uint16_t *w, const float *bias, int act,
                           void *y, int ty, hipStream_t s)
{
    MfGeom m;
    size_t lds = 0;
    if (tx == DT_BF16 && mfma_geom(g, false, m, lds))
        return ty == DT_BF16 ? mfma_t<uint16_t>(m, lds, x, w, bias, act, y, s)
                             : mfma_t<float>(m, lds, x, w, bias, act, y, s);
    if (tx == DT_BF16 && ty == DT_BF16) return fwd_t<uint16_t, uint16_t>(g, x, w, bias, act, y, s);
    if (tx == DT_BF16 && ty == DT_F32) return fwd_t<uint16_t, float>(g, x, w, bias, act, y, s);
    if (tx == DT_F32 && ty == DT_BF16) return fwd_t<float, uint16_t>(g, x, w, bias, act, y, s);
    return fwd_t<float, float>(g, x, w, bias, act, y, s);
}

/* The data gradient of a stride-4 convolution with an 8^3 kernel and
 * padding 4 onto one input channel: the network's last layer (a transposed
 * convolution from the coarse grid to the nodes).  Fine index i = 4 a + r
 * (r = 0..3) receives from coarse points a (tap r + 4) and a + 1 (tap r) in
 * every direction, so one thread owns the 4^3 fine points of block a and
 * reads the 8 coarse values they share once per channel; the weights of a
 * channel (512 taps) are read from LDS as broadcasts.  The direct kernel
 * re-reads every coarse value for each of its fine points. */
constexpr int T4_MAXC = 32;

template <typename TG, typename TO>
__global__ __launch_bounds__(NN_WG) void tconv_s4k8_kernel(const ConvGeom g, const TG *__restrict__ gr,
                                                           const uint16_t *__restrict__ w,
                                                           const float *__restrict__ bias_in, TO *__restrict__ dx)
{
    __shared__ uint16_t wl[T4_MAXC * 512];
    for (int e = threadIdx.x; e < g.co * 512; e += NN_WG) wl[e] = w[e]; /* w[co][0][tz][ty][tx] */
    __syncthreads();
    const int bx = (g.in[2] + 3) / 4, by = (g.in[1] + 3) / 4, bz = (g.in[0] + 3) / 4;
    const int64_t nb = (int64_t)bx * by * bz;
    const int64_t t = (int64_t)blockIdx.x * NN_WG + threadIdx.x;
    if (t >= (int64_t)g.n * nb) return;
    const int n = (int)(t / nb);
    int64_t rem = t - (int64_t)n * nb;
    const int ax = (int)(rem % bx);
    rem /= bx;
    const int ay = (int)(rem % by), az = (int)(rem / by);
    const int64_t ovox = (int64_t)g.out[0] * g.out[1] * g.out[2];
    float acc[4][4][4];
#pragma unroll
    for (int i = 0; i < 64; ++i) acc[i >> 4][(i >> 2) & 3][i & 3] = 0.f;
    for (int co = 0; co < g.co; ++co) {
        const TG *gc = gr + ((int64_t)n * g.co + co) * ovox;
        float gv[2][2][2];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int oz = az + (j >> 2), oy = ay + ((j >> 1) & 1), ox = ax + (j & 1);
            gv[j >> 2][(j >> 1) & 1][j & 1] =
                (oz < g.out[0] && oy < g.out[1] && ox < g.out[2])
                    ? load_f(gc, ((int64_t)oz * g.out[1] + oy) * g.out[2] + ox)
                    : 0.f;
        }
        const uint16_t *wc = wl + co * 512;
#pragma unroll
        for (int rz = 0; rz < 4; ++rz)
#pragma unroll
            for (int ry = 0; ry < 4; ++ry)
#pragma unroll
                for (int rx = 0; rx < 4; ++rx) {
                    float a = acc[rz][ry][rx];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int jz = j >> 2, jy = (j >> 1) & 1, jx = j & 1;
                        /* coarse a (j = 0): tap r + 4; coarse a + 1 (j = 1): tap r */
                        const int tz = rz + 4 * (1 - jz), ty = ry + 4 * (1 - jy), tx = rx + 4 * (1 - jx);
                        a = fmaf(bf16_to_f32(wc[(tz * 8 + ty) * 8 + tx]), gv[jz][jy][jx], a);
                    }
                    acc[rz][ry][rx] = a;
                }
    }
    const float b0 = bias_in ? bias_in[0] : 0.f;
    const int64_t ivox = (int64_t)g.in[0] * g.in[1] * g.in[2];
#pragma unroll
    for (int rz = 0; rz < 4; ++rz)
#pragma unroll
        for (int ry = 0; ry < 4; ++ry)
#pragma unroll
            for (int rx = 0; rx < 4; ++rx) {
                const int iz = 4 * az + rz, iy = 4 * ay + ry, ix = 4 * ax + rx;
                if (iz < g.in[0] && iy < g.in[1] && ix < g.in[2])
                    store_f(dx, (int64_t)n * ivox + ((int64_t)iz * g.in[1] + iy) * g.in[2] + ix, acc[rz][ry][rx] + b0);
            }
}

static bool tconv_s4k8(const ConvGeom &g)
{
    if (g.ci != 1 || g.co < 1 || g.co > T4_MAXC) return false;
    for (int i = 0; i < 3; ++i)
        if (g.k[i] != 8 || g.s[i] != 4 || g.p[i] != 4 || g.d[i] != 1) return false;
    return true;
}

template <typename TG, typename TO>
static hipError_t bwd_data_t(const ConvGeom &g, const void *gr, const uint16_t *w, const float *bias, void *dx,
                             hipStream_t s)
{
    if (tconv_s4k8(g)) {
        const int64_t tot = (int64_t)g.n * ((g.in[0] + 3) / 4) * ((g.in[1] + 3) / 4) * ((g.in[2] + 3) / 4);
        hipLaunchKernelGGL((tconv_s4k8_kernel<TG, TO>), dim3((unsigned)((tot + NN_WG - 1) / NN_WG)), dim3(NN_WG), 0, s,
                           g, (const TG *)gr, w, bias, (TO *)dx);
        return hipGetLastError();
    }
    const int T = g.k[0] * g.k[1] * g.k[2];
    const int64_t tot = (int64_t)g.n * g.in[0] * g.in[1] * g.in[2];
    const unsigned gx = (unsigned)((tot + NN_WG - 1) / NN_WG);
    if (g.ci % 8 == 0) {
        hipLaunchKernelGGL((conv_bwd_data_kernel<TG, TO, 8>), dim3(gx, g.ci / 8), dim3(NN_WG),
                           (size_t)g.co * T * 8 * sizeof(float), s, g, (const TG *)gr, w, bias, (TO *)dx);
    } else {
        hipLaunchKernelGGL((conv_bwd_data_kernel<TG, TO, 1>), dim3(gx, g.ci), dim3(NN_WG),
                           (size_t)g.co * T * sizeof(float), s, g, (const TG *)gr, w, bias, (TO *)dx);
    }
    return hipGetLastError();
}

hipError_t launch_conv_bwd_data(const ConvGeom &g, const void *gr, int tg, const uint16_t *w, const float *bias,
                                void *dx, int tdx, hipStream_t s)
{
    MfGeom m;
    size_t lds = 0;
    if (tg == DT_BF16 && !bias && mfma_geom(g, true, m, lds))
        return tdx == DT_BF16 ? mfma_t<uint16_t>(m, lds, gr, w, nullptr, ACT_NONE, dx, s)
                              : mfma_t<float>(m, lds, gr, w, nullptr, ACT_NONE, dx, s);
    if (tg == DT_BF16 && tdx == DT_BF16) return bwd_data_t<uint16_t, uint16_t>(g, gr, w, bias, dx, s);
    if (tg == DT_BF16 && tdx == DT_F32) return bwd_data_t<uint16_t, float>(g, gr, w, bias, dx, s);
    if (tg == DT_F32 && tdx == DT_BF16) return bwd_data_t<float, uint16_t>(g, gr, w, bias, dx, s);
    return bwd_data_t<float, float>(g, gr, w, bias, dx, s);
}

static bool mfma_geom(const ConvGeom &g, bool flip, MfGeom &m, size_t &lds);

int wgrad_chunks(const ConvGeom &g)
{
    MfGeom m;
    size_t lds = 0;
    if (mfma_geom(g, false, m, lds) && m.K == 3) return MFW_CHUNKS; /* one chunk per matrix-core workgroup */
    const int64_t T = (int64_t)g.k[0] * g.k[1] * g.k[2];
    const int64_t blocks = (int64_t)g.ci * T * (g.co % 8 == 0 ? g.co / 8 : g.co);
    int64_t c = (4096 + blocks - 1) / blocks;
    if (c < 1) c = 1;
    if (c > 64) c = 64;
    return (int)c;
}

template <typename TX, typename TG>
static hipError_t wgrad_t(const ConvGeom &g, const void *x, const void *gr, float *dw, float *db, float *work,
                          hipStream_t s)
{
    const int T = g.k[0] * g.k[1] * g.k[2];
    const int nch = wgrad_chunks(g);
    if (g.co % 8 == 0)
        hipLaunchKernelGGL((conv_bwd_weight_kernel<TX, TG, 8>), dim3(g.ci * T, nch, g.co / 8), dim3(NN_WG), 0, s, g,
                           (const TX *)x, (const TG *)gr, work);
    else
        hipLaunchKernelGGL((conv_bwd_weight_kernel<TX, TG, 1>), dim3(g.ci * T, nch, g.co), dim3(NN_WG), 0, s, g,
                           (const TX *)x, (const TG *)gr, work);
    const int64_t nw = (int64_t)g.co * g.ci * T;
    hipLaunchKernelGGL(conv_wsum_kernel, dim3((unsigned)((nw + NN_WG - 1) / NN_WG)), dim3(NN_WG), 0, s, nw, nch,
                       (const float *)work, dw);
    /* db with the (now consumed) chunk buffer as its partial-sum workspace */
    if (db) return channel_sum_t<TG>(g, gr, db, work, (int64_t)nch * nw, s);
    return hipGetLastError();
}

hipError_t launch_conv_bwd_weight(const ConvGeom &g, const void *x, int tx, const void *gr, int tg, float *dw,
                                  float *db, float *work, hipStream_t s)
{
    MfGeom m;
    size_t lds_fwd = 0;
    if (tx == DT_BF16 && tg == DT_BF16 && mfma_geom(g, false, m, lds_fwd) && m.K == 3) {
        const size_t lds = (size_t)MF_C * MF_PTS * sizeof(uint16_t) + (size_t)m.RMAX * m.SW * MF_C * sizeof(uint16_t) +
                           MF_PTS * sizeof(int);
        if (lds <= MAX_LDS_BYTES) {
            const int T = 27;
            hipLaunchKernelGGL((conv_wgrad_mfma_kernel<3>), dim3(MFW_CHUNKS), dim3(MFW_WG), lds, s, m,
                               (const uint16_t *)x, (const uint16_t *)gr, work, MFW_CHUNKS);
            const int64_t nw = (int64_t)MF_C * MF_C * T;
            hipLaunchKernelGGL(conv_wsum_kernel, dim3((unsigned)((nw + NN_WG - 1) / NN_WG)), dim3(NN_WG), 0, s, nw,
                               MFW_CHUNKS, (const float *)work, dw);
            if (db) return channel_sum_t<uint16_t>(g, gr, db, work, (int64_t)MFW_CHUNKS * nw, s);
            return hipGetLastError();
        }
    }
    if (tx == DT_BF16 && tg == DT_BF16) return wgrad_t<uint16_t, uint16_t>(g, x, gr, dw, db, work, s);
    if (tx == DT_BF16 && tg == DT_F32) return wgrad_t<uint16_t, float>(g, x, gr, dw, db, work, s);
    if (tx == DT_F32 && tg == DT_BF16) return wgrad_t<float, uint16_t>(g, x, gr, dw, db, work, s);
    return wgrad_t<float, float>(g, x, gr, dw, db, work, s);
}

hipError_t launch_act_bwd(int64_t n, const float *dy, const void *y, int ty, float *dz, hipStream_t s)
{
    if (ty == DT_BF16)
        hipLaunchKernelGGL(act_bwd_kernel<uint16_t>, dim3(grid_for(n)), dim3(NN_WG), 0, s, n, dy, (const uint16_t *)y, dz);
    else
        hipLaunchKernelGGL(act_bwd_kernel<float>, dim3(grid_for(n)), dim3(NN_WG), 0, s, n, dy, (const float *)y, dz);
    return hipGetLastError();
}

int mse_blocks(int64_t n)
{
    int64_t b = (n + NN_WG * 8 - 1) / (NN_WG * 8);
    if (b < 1) b = 1;
    if (b > MSE_MAX_BLOCKS) b = MSE_MAX_BLOCKS;
    return (int)b;
}

hipError_t launch_mse(int64_t n, const float *pred, const float *target, float *grad, double *loss, double *work,
                      hipStream_t s)
{
    const int nb = mse_blocks(n);
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(NN_WG), 0, s, n, pred, target, grad, work);
    hipLaunchKernelGGL(mse_sum_kernel, dim3(1), dim3(64), 0, s, nb, n, (const double *)work, loss);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float *th, uint16_t *thb, const float *gr, float *m, float *v, int step, float lr,
                       float b1, float b2, float eps, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(NN_WG), 0, s, n, th, thb, gr, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_convert(int64_t n, const void *in, int tin, void *out, int tout, hipStream_t s)
{
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(NN_WG), 0, s, n, in, tin, out, tout);
    return hipGetLastError();
}

hipError_t launch_features(const FeatGeom &f, const double *logc, const double *b, const double *diag, double *work,
                           uint16_t *out, hipStream_t s)
{
    const int nb = FEAT_NORM_BLOCKS;
    hipLaunchKernelGGL(feat_norm_kernel, dim3(nb), dim3(NN_WG), 0, s, f.n, b, diag, work);
    hipLaunchKernelGGL(feat_kernel, dim3((unsigned)((f.n + NN_WG - 1) / NN_WG)), dim3(NN_WG), 0, s, f, logc, b, diag,
                       (const double *)work, nb, out);
    return hipGetLastError();
}

hipError_t launch_channel_sum(const ConvGeom &g, const void *gr, int tg, float *out, float *work,
                              int64_t work_floats, hipStream_t s)
{
    if (tg == DT_BF16) return channel_sum_t<uint16_t>(g, gr, out, work, work_floats, s);
    return channel_sum_t<float>(g, gr, out, work, work_floats, s);
}

hipError_t launch_normalize(int64_t n, const double *in, double *work, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(sumsq64_kernel, dim3(FEAT_NORM_BLOCKS), dim3(NN_WG), 0, s, n, in, work);
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)((n + NN_WG - 1) / NN_WG)), dim3(NN_WG), 0, s, n, in,
                       (const double *)work, FEAT_NORM_BLOCKS, out);
    return hipGetLastError();
}

}  // namespace mfnn
