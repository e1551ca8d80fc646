/*
 * nn_capi.hip -- C ABI of the warm-start network kernels (include/mfnn.h):
 * host-side validation of every descriptor and size, then the launches.
 */
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/mfnn.h"
#include "nn_kernels.h"

using namespace mfnn;

/* Workspace of mfnn_conv3d_bwd_weight_noalloc: the per-chunk partial weight
 * gradients live in this array instead of a caller buffer.  Each GPU holds
 * its own copy for the life of the process.  Host code never passes the
 * array's name to a kernel (on the host it is a stand-in, not a device
 * address); it passes the device address that hipGetSymbolAddress returned
 * for the current device. */
static __device__ __align__(256) float scratch[MFNN_NOALLOC_WORK_FLOATS];

constexpr int MAX_SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[MAX_SCRATCH_DEVICES];

static thread_local std::string g_nn_err;

static int nn_fail(int code, const std::string &msg)
{
    g_nn_err = msg;
    return code;
}

#define NNCHK(expr)                                                                           \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (void)hipGetLastError(); /* reported here; not left for the caller's next HIP call */ \
            return nn_fail(MFNN_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
        }                                                                                     \
    } while (0)

static bool dtype_ok(int32_t t) { return t == MFNN_BF16 || t == MFNN_F32; }

static int check_desc(const mfnn_conv_desc *d, ConvGeom &g)
{
    if (!d) return nn_fail(MFNN_EINVAL, "null descriptor");
    if (d->n < 1 || d->c_in < 1 || d->c_out < 1) return nn_fail(MFNN_EINVAL, "n, c_in, c_out must be >= 1");
    g.n = d->n;
    g.ci = d->c_in;
    g.co = d->c_out;
    for (int i = 0; i < 3; ++i) {
        if (d->k[i] < 1 || d->k[i] > 8) return nn_fail(MFNN_EINVAL, "kernel size must be in 1..8");
        if (d->stride[i] < 1 || d->dil[i] < 1 || d->pad[i] < 0) return nn_fail(MFNN_EINVAL, "bad stride/dil/pad");
        if (d->in[i] < 1 || d->out[i] < 1) return nn_fail(MFNN_EINVAL, "spatial sizes must be >= 1");
        const int64_t span = (int64_t)d->in[i] + 2 * (int64_t)d->pad[i] - (int64_t)d->dil[i] * (d->k[i] - 1) - 1;
        if (span < 0 || span / d->stride[i] + 1 != d->out[i])
            return nn_fail(MFNN_EINVAL, "out != (in + 2 pad - dil (k - 1) - 1) / stride + 1");
        g.in[i] = d->in[i];
        g.out[i] = d->out[i];
        g.k[i] = d->k[i];
        g.s[i] = d->stride[i];
        g.p[i] = d->pad[i];
        g.d[i] = d->dil[i];
    }
    const int64_t ivox = (int64_t)g.in[0] * g.in[1] * g.in[2], ovox = (int64_t)g.out[0] * g.out[1] * g.out[2];
    if ((int64_t)g.n * g.ci * ivox > ((int64_t)1 << 40) || (int64_t)g.n * g.co * ovox > ((int64_t)1 << 40))
        return nn_fail(MFNN_EINVAL, "tensor too large");
    if ((int64_t)g.n * ivox > ((int64_t)1 << 31) * 256 || (int64_t)g.n * ovox > ((int64_t)1 << 31) * 256)
        return nn_fail(MFNN_EINVAL, "too many points for one launch");
    return MFNN_OK;
}

extern "C" {

const char *mfnn_last_error(void) { return g_nn_err.c_str(); }

int mfnn_conv3d_fwd(const mfnn_conv_desc *desc, const void *x, int32_t x_dtype, const uint16_t *w,
                    const float *bias, int32_t act, void *y, int32_t y_dtype, void *hip_stream)
{
    ConvGeom g{};
    int rc = check_desc(desc, g);
    if (rc) return rc;
    if (!x || !w || !y) return nn_fail(MFNN_EINVAL, "null tensor");
    if (!dtype_ok(x_dtype) || !dtype_ok(y_dtype)) return nn_fail(MFNN_EINVAL, "x and y must be BF16 or F32");
    if (act != MFNN_ACT_NONE && act != MFNN_ACT_LEAKY) return nn_fail(MFNN_EINVAL, "unknown activation");
    const size_t lds = (size_t)g.ci * g.k[0] * g.k[1] * g.k[2] * (g.co % 8 == 0 ? 8 : 1) * sizeof(float);
    if (lds > MAX_LDS_BYTES && !(x_dtype == MFNN_BF16 && mfma_applies(g, false)))
        return nn_fail(MFNN_EINVAL, "layer weights exceed the LDS budget");
    NNCHK(launch_conv_fwd(g, x, x_dtype, w, bias, act, y, y_dtype, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_conv3d_bwd_data(const mfnn_conv_desc *desc, const void *gr, int32_t g_dtype, const uint16_t *w,
                         const float *bias_in, void *dx, int32_t dx_dtype, void *hip_stream)
{
    ConvGeom g{};
    int rc = check_desc(desc, g);
    if (rc) return rc;
    if (!gr || !w || !dx) return nn_fail(MFNN_EINVAL, "null tensor");
    if (!dtype_ok(g_dtype) || !dtype_ok(dx_dtype)) return nn_fail(MFNN_EINVAL, "g and dx must be BF16 or F32");
    const size_t lds = (size_t)g.co * g.k[0] * g.k[1] * g.k[2] * (g.ci % 8 == 0 ? 8 : 1) * sizeof(float);
    if (lds > MAX_LDS_BYTES && !(g_dtype == MFNN_BF16 && !bias_in && mfma_applies(g, true)))
        return nn_fail(MFNN_EINVAL, "layer weights exceed the LDS budget");
    NNCHK(launch_conv_bwd_data(g, gr, g_dtype, w, bias_in, dx, dx_dtype, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int64_t mfnn_conv3d_bwd_weight_work(const mfnn_conv_desc *desc)
{
    ConvGeom g{};
    if (check_desc(desc, g)) return -1;
    return (int64_t)wgrad_chunks(g) * g.co * g.ci * g.k[0] * g.k[1] * g.k[2];
}

int mfnn_conv3d_bwd_weight(const mfnn_conv_desc *desc, const void *x, int32_t x_dtype, const void *gr,
                           int32_t g_dtype, float *dw, float *db, float *work, int64_t work_floats,
                           void *hip_stream)
{
    ConvGeom g{};
    int rc = check_desc(desc, g);
    if (rc) return rc;
    if (!x || !gr || !dw || !work) return nn_fail(MFNN_EINVAL, "null tensor");
    if (!dtype_ok(x_dtype) || !dtype_ok(g_dtype)) return nn_fail(MFNN_EINVAL, "x and g must be BF16 or F32");
    if (work_floats < mfnn_conv3d_bwd_weight_work(desc)) return nn_fail(MFNN_EINVAL, "work buffer too small");
    NNCHK(launch_conv_bwd_weight(g, x, x_dtype, gr, g_dtype, dw, db, work, (hipStream_t)hip_stream));
    return MFNN_OK;
}

/* Device address of the current device's copy of the scratch array, looked
 * up once per device (on the first call made with that device current). */
static int scratch_of_current_device(float **out)
{
    int dev = -1;
    NNCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_SCRATCH_DEVICES) return nn_fail(MFNN_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        float *p = nullptr;
        NNCHK(hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)));
        if (!p) return nn_fail(MFNN_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MFNN_OK;
}

int mfnn_conv3d_bwd_weight_noalloc(const mfnn_conv_desc *desc, const void *x, int32_t x_dtype, const void *gr,
                                   int32_t g_dtype, float *dw, float *db, void *hip_stream)
{
    ConvGeom g{};
    int rc = check_desc(desc, g);
    if (rc) return rc;
    if (!x || !gr || !dw) return nn_fail(MFNN_EINVAL, "null tensor");
    if (!dtype_ok(x_dtype) || !dtype_ok(g_dtype)) return nn_fail(MFNN_EINVAL, "x and g must be BF16 or F32");
    const int64_t need = mfnn_conv3d_bwd_weight_work(desc);
    if (need < 0 || need > MFNN_NOALLOC_WORK_FLOATS)
        return nn_fail(MFNN_EINVAL, "layer needs " + std::to_string(need) +
                                        " floats of weight-gradient workspace; the allocation-free entry point has " +
                                        std::to_string((long long)MFNN_NOALLOC_WORK_FLOATS));
    float *work = nullptr;
    rc = scratch_of_current_device(&work);
    if (rc) return rc;
    NNCHK(launch_conv_bwd_weight(g, x, x_dtype, gr, g_dtype, dw, db, work, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_act_bwd(int64_t n, const float *dy, const void *y, int32_t y_dtype, int32_t act, float *dz,
                 void *hip_stream)
{
    if (n < 0 || !dy || !y || !dz) return nn_fail(MFNN_EINVAL, "bad argument");
    if (!dtype_ok(y_dtype)) return nn_fail(MFNN_EINVAL, "y must be BF16 or F32");
    if (act != MFNN_ACT_LEAKY) return nn_fail(MFNN_EINVAL, "only the leaky ReLU has a backward map");
    if (n == 0) return MFNN_OK;
    NNCHK(launch_act_bwd(n, dy, y, y_dtype, dz, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_mse(int64_t n, const float *pred, const float *target, float *grad, double *loss, double *work,
             void *hip_stream)
{
    if (n < 1 || !pred || !target || !grad || !loss || !work) return nn_fail(MFNN_EINVAL, "bad argument");
    NNCHK(launch_mse(n, pred, target, grad, loss, work, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_mse_loss(int64_t n, const float *pred, const float *target, float *grad, double *loss, double *work,
                  void *hip_stream)
{
    return mfnn_mse(n, pred, target, grad, loss, work, hip_stream);
}

int mfnn_adam_step(int64_t n, float *theta, uint16_t *theta_bf16, const float *g, float *m, float *v, int32_t step,
                   float lr, float beta1, float beta2, float eps, void *hip_stream)
{
    return mfnn_adam(n, theta, theta_bf16, g, m, v, step, lr, beta1, beta2, eps, hip_stream);
}

int mfnn_adam(int64_t n, float *theta, uint16_t *theta_bf16, const float *g, float *m, float *v, int32_t step,
              float lr, float beta1, float beta2, float eps, void *hip_stream)
{
    if (n < 0 || !theta || !g || !m || !v) return nn_fail(MFNN_EINVAL, "bad argument");
    if (step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return nn_fail(MFNN_EINVAL, "bad hyper-parameter");
    if (n == 0) return MFNN_OK;
    NNCHK(launch_adam(n, theta, theta_bf16, g, m, v, step, lr, beta1, beta2, eps, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_convert(int64_t n, const void *in, int32_t in_dtype, void *out, int32_t out_dtype, void *hip_stream)
{
    if (n < 0 || !in || !out) return nn_fail(MFNN_EINVAL, "bad argument");
    const auto ok = [](int32_t t) { return t == MFNN_BF16 || t == MFNN_F32 || t == MFNN_F64; };
    if (!ok(in_dtype) || !ok(out_dtype)) return nn_fail(MFNN_EINVAL, "unknown dtype");
    if (n == 0) return MFNN_OK;
    NNCHK(launch_convert(n, in, in_dtype, out, out_dtype, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_features(const int32_t cells[3], int32_t k, const double *log_coeff, const double *b,
                  const double *diag, double *work, uint16_t *out, void *hip_stream)
{
    if (!cells || !log_coeff || !b || !diag || !work || !out) return nn_fail(MFNN_EINVAL, "null argument");
    if (k < 1 || k > 8) return nn_fail(MFNN_EINVAL, "degree must be in 1..8");
    FeatGeom f{};
    f.k = k;
    f.n = 1;
    for (int d = 0; d < 3; ++d) {
        if (cells[d] < 1) return nn_fail(MFNN_EINVAL, "cells must be >= 1");
        f.cells[d] = cells[d];
        f.n *= (int64_t)cells[d] * k + 1;
    }
    if (f.n > ((int64_t)1 << 36)) return nn_fail(MFNN_EINVAL, "mesh too large");
    NNCHK(launch_features(f, log_coeff, b, diag, work, out, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_channel_sum(int32_t n, int32_t c, const int32_t spatial[3], const void *g, int32_t g_dtype, float *out,
                     void *hip_stream)
{
    return mfnn_channel_sum_work(n, c, spatial, g, g_dtype, out, nullptr, 0, hip_stream);
}

int mfnn_channel_sum_work(int32_t n, int32_t c, const int32_t spatial[3], const void *g, int32_t g_dtype,
                          float *out, float *work, int64_t work_floats, void *hip_stream)
{
    if (work_floats < 0 || (work_floats > 0 && !work)) return nn_fail(MFNN_EINVAL, "bad workspace");
    if (n < 1 || c < 1 || !spatial || !g || !out) return nn_fail(MFNN_EINVAL, "bad argument");
    if (!dtype_ok(g_dtype)) return nn_fail(MFNN_EINVAL, "g must be BF16 or F32");
    ConvGeom geo{};
    geo.n = n;
    geo.co = c;
    for (int d = 0; d < 3; ++d) {
        if (spatial[d] < 1) return nn_fail(MFNN_EINVAL, "spatial sizes must be >= 1");
        geo.out[d] = spatial[d];
    }
    NNCHK(launch_channel_sum(geo, g, g_dtype, out, work, work_floats, (hipStream_t)hip_stream));
    return MFNN_OK;
}

int mfnn_normalize(int64_t n, const double *in, double *work, float *out, void *hip_stream)
{
    if (n < 1 || !in || !work || !out) return nn_fail(MFNN_EINVAL, "bad argument");
    NNCHK(launch_normalize(n, in, work, out, (hipStream_t)hip_stream));
    return MFNN_OK;
}

}  // extern "C"
