/* nn_kernels.h -- launch wrappers of the warm-start network kernels. */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfnn {

enum DType : int { DT_BF16 = 0, DT_F32 = 1, DT_F64 = 2 };
enum Act : int { ACT_NONE = 0, ACT_LEAKY = 1 };
constexpr float LEAKY_SLOPE = 0.1f;
constexpr int MSE_MAX_BLOCKS = 1024;
constexpr int FEAT_NORM_BLOCKS = 1024;
constexpr size_t MAX_LDS_BYTES = 65536;

/* Convolution geometry, spatial order (D, H, W) = (z, y, x). */
struct ConvGeom {
    int32_t n, ci, co;
    int32_t in[3], out[3];
    int32_t k[3], s[3], p[3], d[3];
};

/* Node lattice of the solver mesh: (cells[d] * k + 1) nodes per direction. */
struct FeatGeom {
    int32_t cells[3], k;
    int64_t n;
};

/* the layer runs on the matrix cores with BF16 input (forward map; flip:
 * the data gradient without bias) */
bool mfma_applies(const ConvGeom &g, bool flip);
hipError_t launch_conv_fwd(const ConvGeom &g, const void *x, int tx, const uint16_t *w, const float *bias, int act,
                           void *y, int ty, hipStream_t s);
hipError_t launch_conv_bwd_data(const ConvGeom &g, const void *gr, int tg, const uint16_t *w, const float *bias,
                                void *dx, int tdx, hipStream_t s);
int wgrad_chunks(const ConvGeom &g);
hipError_t launch_conv_bwd_weight(const ConvGeom &g, const void *x, int tx, const void *gr, int tg, float *dw,
                                  float *db, float *work, hipStream_t s);
hipError_t launch_act_bwd(int64_t n, const float *dy, const void *y, int ty, float *dz, hipStream_t s);
int mse_blocks(int64_t n);
hipError_t launch_mse(int64_t n, const float *pred, const float *target, float *grad, double *loss, double *work,
                      hipStream_t s);
hipError_t launch_adam(int64_t n, float *th, uint16_t *thb, const float *gr, float *m, float *v, int step, float lr,
                       float b1, float b2, float eps, hipStream_t s);
hipError_t launch_convert(int64_t n, const void *in, int tin, void *out, int tout, hipStream_t s);
hipError_t launch_features(const FeatGeom &f, const double *logc, const double *b, const double *diag, double *work,
                           uint16_t *out, hipStream_t s);

/* out[c] = sum over n and the spatial points of channel c (g.co channels, g.out points) */
/* work: NULL (one block per channel) or work_floats >= 2 co floats of scratch
 * (up to CSUM_MAX_BLOCKS blocks per channel, partial sums in work) */
constexpr int CSUM_MAX_BLOCKS = 512;
hipError_t launch_channel_sum(const ConvGeom &g, const void *gr, int tg, float *out, float *work, int64_t work_floats,
                              hipStream_t s);
hipError_t launch_normalize(int64_t n, const double *in, double *work, float *out, hipStream_t s);

}  // namespace mfnn
