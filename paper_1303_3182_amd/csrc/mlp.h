// The selector network's kernels (mlp.hip).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

namespace tqr {

constexpr int kMlpHidden = 64;
constexpr int kMlpFeatures = 9;
constexpr int kMlpParams = kMlpHidden * kMlpFeatures + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden + 1;

size_t mlp_work_bytes(int64_t B);
hipError_t mlp_forward(const float *w, const float *X, int64_t B, float *Y, hipStream_t s);
hipError_t mlp_grad(const float *w, const float *X, const float *T, int64_t B, float *grad, float *loss, void *work,
                    hipStream_t s);
hipError_t mlp_adam(float *w, const float *g, float *m1, float *m2, int64_t t, float lr, hipStream_t s);
hipError_t mlp_zero(float *x, int64_t n, hipStream_t s);

}  // namespace tqr
