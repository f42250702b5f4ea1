// One Adam update (Kingma and Ba 2015, with bias correction), shared by the
// plain Adam pass over an array and by the projection backward's fused
// update, so both produce the same bits for the same gradient.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "wsr_internal.h"

namespace wsr {

struct AdamStep {
  float b1, b2, eps;
  float bc1, bc2;  // 1 - b1^step, 1 - b2^step
};

inline AdamStep make_adam_step(int32_t step, float b1, float b2, float eps) {
  AdamStep s;
  s.b1 = b1;
  s.b2 = b2;
  s.eps = eps;
  s.bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), step));
  s.bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), step));
  return s;
}

// m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2 (in place); returns the
// parameter p - lr (m / bc1) / (sqrt(v / bc2) + eps).
__device__ __forceinline__ float adam_update(float p, float g, float& m, float& v, float lr, const AdamStep& s) {
  m = fmaf(s.b1, m, (1.f - s.b1) * g);
  v = fmaf(s.b2, v, (1.f - s.b2) * g * g);
  return p - lr * (m / s.bc1) / (sqrtf(v / s.bc2) + s.eps);
}

// One Adam step of the per-Gaussian parameters fused into the projection
// backward: the moments m and v in the gradients' layout (their globals
// fields unused) and one learning rate per group (means, log-scales,
// quaternions, SH degree 0, higher SH degrees, logit, v_i).
struct FusedAdam {
  wsr_grads m, v;
  float lr[7];
  AdamStep step;
};

// launch_project_bwd with the update fused in (FP32 storage): the scene's
// per-Gaussian arrays are updated in place instead of gradients written;
// grad_globals receives the gradient of the global parameters.
hipError_t launch_project_bwd_adam(const wsr_scene* sc, const wsr_params* P, const float* globals,
                                   const Layout& L, void* ws, const void* pairs, int64_t capacity,
                                   const FusedAdam& f, float* grad_globals, float* out_grad2d, hipStream_t st);

}  // namespace wsr
