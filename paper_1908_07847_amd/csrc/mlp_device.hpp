// Device-side helpers shared by the libmlp kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.h"

namespace mlpk {

constexpr int kWave = 64;
constexpr int kLayerMaxOut = 16;  // outputs supported by the generic layer kernels

// Equation 1 of the paper: sigma(z) = 1 / (1 + e^-z).  expf is the accurate
// device exponential; exp(-z) overflowing to +inf gives 0, the right limit.
__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// theta <- theta - lr*g.  With a compensation term c (Kahan summation of the
// update stream) the low-order bits lost when a small step is added to a
// larger weight are carried to the next update instead of being dropped.
__device__ __forceinline__ void gd_update(float &w, float &c, float lr, float g, bool compensated) {
  if (compensated) {
    float y = -lr * g - c;
    float t = w + y;
    c = (t - w) - y;
    w = t;
  } else {
    w = w - lr * g;
  }
}

// Sum over the 64 lanes of a wave, fixed butterfly order (deterministic).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace mlpk

// Launch wrappers implemented in the .hip files and used by the host API.
namespace mlph {

// Small-network trainer: one workgroup per net, all epochs in one launch.
// items == nullptr means a single net described by `one`.
size_t small_lds_bytes(int n_rows, int n_hidden, int n_in);
hipError_t launch_small_train(const mlp_batch_item *items, mlp_batch_item one, int n_nets,
                              int n_in, int n_out, int max_rows, int max_hidden, const float *X,
                              const float *T, float *theta, float *comp, int epochs,
                              float *loss_hist, hipStream_t s);

// Generic layer kernels (any sizes) for mlp_forward / mlp_backward / mlp_step.
hipError_t launch_forward(int64_t n, int D, int H, int K, const float *X, mlp_params p, float *A,
                          float *Y, hipStream_t s);
hipError_t launch_backward(int64_t n, int D, int H, int K, const float *X, const float *A,
                           const float *Y, const float *dY, const float *T, mlp_params p,
                           mlp_params g, float *dX, float *loss, float *ws, hipStream_t s);
hipError_t launch_step(int D, int H, int K, mlp_params p, mlp_params g, float *comp, float lr,
                       hipStream_t s);

}  // namespace mlph
