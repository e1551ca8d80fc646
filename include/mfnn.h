/*
 * mfnn.h -- C ABI of the learned warm start's network kernels (gfx950).
 *
 * A small 3D convolutional network maps the coefficient field and the
 * right-hand side of the Poisson problem to an initial guess x0 for the CG
 * solver of mfcg.h; it is trained on solutions the solver produced.  The
 * paper has no learned component: this is an extension around its method,
 * judged only by the CG residual (the iterations the guess saves).
 *
 * Conventions (all functions):
 *   - tensors are device pointers in NCDHW order (W fastest), contiguous;
 *     the spatial order (D, H, W) = (z, y, x) matches the x-fastest
 *     lexicographic node order of mfcg vectors;
 *   - element types are selected per argument: MFNN_BF16 (uint16_t bit
 *     patterns of bfloat16), MFNN_F32, MFNN_F64 (mfnn_convert only);
 *   - weights are BF16 [c_out][c_in][kd][kh][kw]; biases, weight
 *     gradients and optimiser state are FP32; every product is accumulated
 *     in FP32;
 *   - every reduction is summed in a fixed order (bitwise reproducible);
 *   - calls are stream-ordered on hip_stream (a hipStream_t, NULL: the
 *     default stream) and do not synchronise; the caller owns every buffer;
 *   - return 0 (MFNN_OK) or MFNN_EINVAL (bad descriptor, sizes or types,
 *     detected on the host before any launch) or MFNN_EHIP (a launch
 *     failed).
 */
#ifndef MFNN_H
#define MFNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MFNN_OK = 0, MFNN_EINVAL = -1, MFNN_EHIP = -3 };
enum { MFNN_BF16 = 0, MFNN_F32 = 1, MFNN_F64 = 2 };
enum { MFNN_ACT_NONE = 0, MFNN_ACT_LEAKY = 1 /* a(z) = z for z > 0, 0.1 z otherwise */ };

/* Convolution y[n,co,o] = b[co] + sum_{ci,t} w[co,ci,t] x[n,ci,o*s - p + t*d]
 * (zero padding), per direction (D, H, W):
 *   out = (in + 2 p - d (k - 1) - 1) / s + 1   (must hold exactly).
 * Limits: n, c_in, c_out >= 1; k in 1..8; s, d >= 1; p >= 0; the layer's
 * weights as FP32 (c_in * k^3 * 8 floats for the forward map, c_out * k^3 * 8
 * for the backward-data map; 8 becomes 1 when the channel count is not a
 * multiple of 8) fit in 64 KiB of LDS. */
typedef struct {
    int32_t n, c_in, c_out;
    int32_t in[3], out[3];
    int32_t k[3], stride[3], pad[3], dil[3];
} mfnn_conv_desc;

/* y = act(conv(x, w) + bias).  x: [n][c_in][in] (x_dtype BF16 or F32);
 * bias: c_out floats or NULL; y: [n][c_out][out] (y_dtype BF16 or F32).
 * A layer with c_in = c_out = 32, stride 1 and a cubic kernel (k <= 5,
 * the same dilation and padding in every direction) and BF16 x runs as an
 * implicit GEMM on the BF16 matrix cores (FP32 accumulation); the others,
 * or those whose staging would not fit 64 KiB of LDS, as direct
 * convolutions.  Both give the products exactly and sum them in FP32. */
int mfnn_conv3d_fwd(const mfnn_conv_desc *desc, const void *x, int32_t x_dtype, const uint16_t *w,
                    const float *bias, int32_t act, void *y, int32_t y_dtype, void *hip_stream);

/* dx = conv(., w)^T g (+ bias_in[ci]): the adjoint of the convolution in x
 * (backward data), which is also the forward map of a transposed
 * convolution with bias_in as its bias.  g: [n][c_out][out] (BF16 or F32);
 * bias_in: c_in floats or NULL; dx: [n][c_in][in] (BF16 or F32).  With
 * BF16 g, no bias_in and a layer of the matrix-core shape above with
 * symmetric padding (2 p = d (k - 1)) it runs on the matrix cores as the
 * forward convolution of g with the flipped, transposed kernel. */
int mfnn_conv3d_bwd_data(const mfnn_conv_desc *desc, const void *g, int32_t g_dtype, const uint16_t *w,
                         const float *bias_in, void *dx, int32_t dx_dtype, void *hip_stream);

/* dw[co,ci,t] = sum_{n,o} g[n,co,o] x[n,ci,o*s - p + t*d] and
 * db[co] = sum_{n,o} g[n,co,o] (db may be NULL).  x: [n][c_in][in], g:
 * [n][c_out][out] (each BF16 or F32); dw: FP32 [c_out][c_in][k^3];
 * work: device scratch of at least mfnn_conv3d_bwd_weight_work(desc) floats. */
int mfnn_conv3d_bwd_weight(const mfnn_conv_desc *desc, const void *x, int32_t x_dtype, const void *g,
                           int32_t g_dtype, float *dw, float *db, float *work, int64_t work_floats,
                           void *hip_stream);
int64_t mfnn_conv3d_bwd_weight_work(const mfnn_conv_desc *desc);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): mfnn_conv3d_bwd_weight with the workspace taken from a
 * library-owned device array of MFNN_NOALLOC_WORK_FLOATS floats (4 MiB), one
 * per GPU, held until the process ends.  The call allocates nothing and
 * gives the same dw and db as mfnn_conv3d_bwd_weight.  Returns MFNN_EINVAL
 * (before any launch) when mfnn_conv3d_bwd_weight_work(desc) exceeds
 * MFNN_NOALLOC_WORK_FLOATS.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams, or host threads without
 * ordering) race and give wrong gradients; calls ordered on one stream are
 * safe.  No part of the array needs to start at any value. */
#define MFNN_NOALLOC_WORK_FLOATS (1 << 20)
int mfnn_conv3d_bwd_weight_noalloc(const mfnn_conv_desc *desc, const void *x, int32_t x_dtype, const void *g,
                                   int32_t g_dtype, float *dw, float *db, void *hip_stream);

/* dz = dy * a'(z), with a'(z) taken from the activation's output y
 * (the leaky ReLU keeps the sign): dz_i = dy_i if y_i > 0 else 0.1 dy_i. */
int mfnn_act_bwd(int64_t n, const float *dy, const void *y, int32_t y_dtype, int32_t act, float *dz,
                 void *hip_stream);

/* loss = mean((pred - target)^2) into *loss (one device double),
 * grad = 2 (pred - target) / n.  work: device scratch of 1024 doubles. */
int mfnn_mse(int64_t n, const float *pred, const float *target, float *grad, double *loss, double *work,
             void *hip_stream);

/* mfnn_mse under the name of the library's interface summary. */
int mfnn_mse_loss(int64_t n, const float *pred, const float *target, float *grad, double *loss, double *work,
                  void *hip_stream);

/* One Adam step (Kingma and Ba, 2015) with bias correction for step >= 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps);
 * theta_bf16 (may be NULL) receives theta rounded to BF16. */
int mfnn_adam(int64_t n, float *theta, uint16_t *theta_bf16, const float *g, float *m, float *v, int32_t step,
              float lr, float beta1, float beta2, float eps, void *hip_stream);
/* mfnn_adam under the name of the library's interface summary. */
int mfnn_adam_step(int64_t n, float *theta, uint16_t *theta_bf16, const float *g, float *m, float *v, int32_t step,
                   float lr, float beta1, float beta2, float eps, void *hip_stream);

/* out[i] = in[i] converted (BF16 / F32 / F64; to BF16 by rounding to
 * nearest even). */
int mfnn_convert(int64_t n, const void *in, int32_t in_dtype, void *out, int32_t out_dtype, void *hip_stream);

/* Input channels of the network on the node lattice of an mfcg mesh with
 * cells[3] cells and degree k (n = prod(cells[d] k + 1) nodes), BF16
 * [3][n]:
 *   channel 0: mean of log a over the cells that touch the node
 *              (log_coeff: device, one double per cell, x fastest);
 *   channel 1: b / rms(b);   channel 2: (b / diag) / rms(b / diag)
 *   (b: load vector, diag: diag(A), device doubles in lexicographic order).
 * work: device scratch of 2048 doubles. */
int mfnn_features(const int32_t cells[3], int32_t k, const double *log_coeff, const double *b,
                  const double *diag, double *work, uint16_t *out, void *hip_stream);

/* out[c] = sum over the n samples and all spatial points of channel c of
 * g ([n][c][spatial], BF16 or F32): the bias gradient of a layer whose
 * output gradient is g (e.g. a transposed convolution's bias). */
int mfnn_channel_sum(int32_t n, int32_t c, const int32_t spatial[3], const void *g, int32_t g_dtype, float *out,
                     void *hip_stream);
/* The same with a caller workspace of work_floats floats (device): the
 * sum of each channel is then spread over up to work_floats / c (at most
 * 512) blocks whose partial sums are added in a fixed order.  work = NULL
 * or work_floats < 2 c: one block per channel, as mfnn_channel_sum. */
int mfnn_channel_sum_work(int32_t n, int32_t c, const int32_t spatial[3], const void *g, int32_t g_dtype,
                          float *out, float *work, int64_t work_floats, void *hip_stream);

/* out = in / rms(in), rms(in) = sqrt(sum in_i^2 / n) (0 if in = 0): the
 * scale-free training target built from a solver solution (FP64 in, FP32
 * out).  work: device scratch of 1024 doubles. */
int mfnn_normalize(int64_t n, const double *in, double *work, float *out, void *hip_stream);

/* Message of the last error on the calling thread. */
const char *mfnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MFNN_H */
