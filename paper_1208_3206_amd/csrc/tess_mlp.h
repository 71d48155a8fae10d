// Refinement network: constants, parameter layout and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tess {
namespace mlp {

constexpr int kWidth = 128;   // hidden width (and number of Fourier features)
constexpr int kFreq = 64;     // Fourier frequencies: features sin and cos of each
constexpr int kDepth = 4;     // hidden layers
constexpr int kSlice = 64;    // batch rows per weight-gradient partial (LDS: 2 x 128 x 72 bf16)
constexpr int kOutPart = 1 + 3 * kWidth + 3;  // loss, dW5, db5 per output block

// Flat FP32 parameter vector: W1 (128 x 128, row = output), b1, ..., W4, b4,
// W5 (3 x 128), b5.
constexpr int64_t kLayerParams = (int64_t)kWidth * kWidth + kWidth;
constexpr int64_t kOffW5 = kDepth * kLayerParams;
constexpr int64_t kOffB5 = kOffW5 + 3 * kWidth;
constexpr int64_t kParams = kOffB5 + 3;
static_assert(kParams == 66435, "parameter count");
__host__ __device__ constexpr int64_t param_offset_W(int l) { return l * kLayerParams; }
__host__ __device__ constexpr int64_t param_offset_b(int l) { return l * kLayerParams + (int64_t)kWidth * kWidth; }

hipError_t launch_rff(const float *q, int64_t n, const float *B, __bf16 *X, hipStream_t s);
hipError_t launch_layer_fwd(const __bf16 *X, int64_t n, const __bf16 *W, const float *b, float *Z,
                            __bf16 *H, hipStream_t s);
hipError_t launch_layer_bwd_data(const __bf16 *dZ, int64_t n, const __bf16 *WT, const float *Zprev,
                                 __bf16 *dZprev, hipStream_t s);
hipError_t launch_grad_w(const __bf16 *dZ, const __bf16 *H, int64_t n, float *part, hipStream_t s);
hipError_t launch_reduce(const float *part, int64_t slices, int64_t stride, int64_t count, float *out,
                         hipStream_t s);
hipError_t launch_out_fwd(const __bf16 *H, int64_t n, const float *W5, const float *b5, float *pred,
                          hipStream_t s);
hipError_t launch_out_bwd(const float *pred, const float *target, int64_t n, const __bf16 *H,
                          const float *Z, const float *W5, __bf16 *dZ, float *part, hipStream_t s);
int64_t out_blocks(int64_t n);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, int64_t count, double lr, double b1,
                       double b2, double eps, int t, hipStream_t s);
hipError_t launch_cast_weights(const float *master, __bf16 *Wb, __bf16 *WTb, hipStream_t s);
// Inference: pred[n][3] from q[n][3] in one pass (features, hidden layers
// and output layer per 16-sample tile in registers; bf16 operands rounded
// from the FP32 master parameters, FP32 accumulation).
hipError_t launch_mlp_infer(const float *q, int64_t n, const float *B, const float *master, float *pred,
                            hipStream_t s);

}  // namespace mlp
}  // namespace tess

namespace tess {
namespace mlp {
hipError_t launch_gather_batch(const float *x, const float *y, const float *z, const int dims[3],
                               const double box[3], uint64_t seed, uint64_t step, int64_t nb, float *q,
                               float *target, hipStream_t s);
hipError_t launch_fine_q(int64_t first, int64_t n, const int fdims[3], float *q, hipStream_t s);
hipError_t launch_place_mlp(const float *cx, const float *cy, const float *cz, const int cdims[3], int r,
                            int64_t first, int64_t n, const float *q, const float *pred,
                            const double box[3], const int fdims[3], float *fx, float *fy, float *fz,
                            hipStream_t s);
// Residuals x - (q + s(q)) L of the network at coarse tracers first..first+n-1.
hipError_t launch_coarse_residual(const float *cx, const float *cy, const float *cz, int64_t first, int64_t n,
                                  const float *q, const float *pred, const double box[3], float *rx, float *ry,
                                  float *rz, hipStream_t s);
// Fine positions first..first+n-1: (q + s(q)) L plus the coarse residuals
// interpolated over the containing coarse tetrahedron.
hipError_t launch_place_hybrid(const float *cx, const float *cy, const float *cz, const float *rx,
                               const float *ry, const float *rz, const int cdims[3], int r, int64_t first,
                               int64_t n, const float *q, const float *pred, const double box[3], float *fx,
                               float *fy, float *fz, hipStream_t s);
hipError_t launch_place_linear(const float *cx, const float *cy, const float *cz, const int cdims[3], int r,
                               const double box[3], float *fx, float *fy, float *fz, hipStream_t s);
}  // namespace mlp
}  // namespace tess
