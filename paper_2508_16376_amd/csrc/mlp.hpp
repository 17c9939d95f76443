// Load predictor kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"

namespace riros {

constexpr int kMlpFeatures = 6;
constexpr int kMlpParams = 4673;                  // 6-64-64-1
constexpr int kMlpWeights = kMlpParams + 2 * 6;   // + normalisation mean, std

struct MlpHyper {
    float lr, beta1, beta2, eps;
};

hipError_t launch_features(const DevDesign& d, const GoldenView& gw, const float4* nodefeat,
                           const riros_fault* faults, uint32_t F, float* out, hipStream_t s);
hipError_t mlp_norm_stats(const float* x, uint32_t S, float* wts, hipStream_t s);
hipError_t mlp_forward(const float* wts, const float* x, uint32_t S, float* out, hipStream_t s);
size_t mlp_partial_floats(uint32_t B);
// One minibatch: gradient (grad_out != NULL: store it, no update) or Adam step.
hipError_t mlp_step(float* wts, const float* x, const float* y, uint32_t B, float* partial, float* loss_part,
                    float* m, float* v, float* grad_out, float* loss_out, uint32_t step, const MlpHyper& h,
                    hipStream_t s);

}  // namespace riros
