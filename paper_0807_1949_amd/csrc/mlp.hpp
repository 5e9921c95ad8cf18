// Learned impedance model: constants and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "vtm_internal.hpp"

namespace vtm {

constexpr int kTrain = 64 * kNumFeatures + 64 + 64 * 64 + 64 + 64 + 1;  // trainable parameters
constexpr int kParams = 2 * kNumFeatures + kTrain;                        // + input mean and std

int mlp_grid(int64_t n);
void launch_mlp_predict(const float *P, const float *X, int64_t n, float *y, hipStream_t st);
void launch_z_from_pred(const float *y, const double *avv, int64_t n, double lo, double hi, double *z, hipStream_t st);
// g[0..kTrain) = gradient of (1/n) sum (y - label)^2 times (scale * n), g[kTrain] = sum of squared errors
void launch_mlp_grad(const float *P, const float *X, const float *Y, const int64_t *idx, int64_t row0, int64_t n,
                     float scale, float *part, int nparts, float *g, hipStream_t st);
void launch_adam(float *P, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, float c1,
                 float c2, hipStream_t st);

}  // namespace vtm
