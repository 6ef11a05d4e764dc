// Host-side interface of the closure kernels (closure.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ops.hpp"

namespace lbrr {

constexpr int kMlpNParam = 6723;  // W1 64x36, b1, W2 64x64, b2, W3 3x64, b3
constexpr int kMlpNNorm = 78;     // x_mean 36, x_std 36, y_mean 3, y_std 3
constexpr int kMlpNPacked = 8768; // BF16 weights, padded rows (layout in mlp.hpp)
constexpr int kMlpNRegImage = 18 * 64 * 8;  // the fused step's weight operands in lane order (closure.hip)
constexpr int kMlpIn = 36;

hipError_t closure_step(int order, int storage, const void* src, void* dst, const StepArgs& a,
                        const uint16_t* packed, const float* params, const float* norm, hipStream_t s);
hipError_t closure_features(int storage, const void* src, float* m, const StepArgs& a, const double* a_target,
                            double plain_weight, float* feat, float* lab, hipStream_t s);
hipError_t closure_coarsen(int dtype, const void* rho, const void* u, const void* pi1, int nfx, int nfy, int F,
                           double alpha, double beta, double* rho_c, double* u_c, double* pi1_c, hipStream_t s);
hipError_t mlp_pack(const float* params, uint16_t* packed, hipStream_t s);
// packed weights (kMlpNPacked) followed by the fused step's register image (kMlpNRegImage)
hipError_t mlp_pack_step(const float* params, uint16_t* packed_and_image, hipStream_t s);
hipError_t mlp_infer(const float* x, int64_t n, const uint16_t* packed, const float* params, const float* norm,
                     float* y, hipStream_t s);
int mlp_train_blocks(int batch);
hipError_t column_stats(const float* x, int64_t n, int dim, float* mean, float* sd, hipStream_t s);
hipError_t mlp_gradient(const float* x, const float* t, int64_t nrows, const int* idx, int batch, const uint16_t* packed,
                        const float* params, const float* norm, float* gpart, float* lpart, float* grad, float* loss,
                        hipStream_t s);
hipError_t mlp_adam(float* p, float* m, float* v, const float* g, long long step, float lr, float b1, float b2,
                    float eps, hipStream_t s);

}  // namespace lbrr
