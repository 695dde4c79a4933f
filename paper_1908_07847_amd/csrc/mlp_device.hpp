// Device-side helpers shared by the libmlp kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.h"

namespace mlpk {

constexpr int kWave = 64;
constexpr int kLayerMaxOut = 16;  // outputs supported by the generic layer kernels

// Logistic sigmoid (Equation 1) from the hardware base-2 exponential and
// reciprocal.  e^-z = 2^(-z log2 e).  Published methods used:
//  - log2 e held as a two-part constant, a high part plus its tail, in the
//    manner of Cody and Waite's argument reduction (Cody & Waite, "Software
//    Manual for the Elementary Functions", 1980);
//  - the rounding error of the product -z * L_HI obtained exactly with one
//    FMA, the error-free transformation TwoProductFMA (Ogita, Rump & Oishi,
//    "Accurate sum and dot product", SIAM J. Sci. Comput. 2005);
//  - 2^(th + tl) = 2^th (1 + tl ln 2) to first order in the small tail tl;
//  - one Newton-Raphson iteration r <- r + r (1 - d r) on the hardware
//    reciprocal of d = 1 + e^-z.
// The exponent so keeps ~48 bits and the result is within a few float ulps
// of the exact sigmoid (checked against float64 in the tests).  For
// z < -87 the exponent is clamped at 2^126 (sigma ~ 1e-38 instead of 0).
__device__ __forceinline__ float sigmoid_e(float z, float &e_out) {
  const float L_HI = 1.44269502162933349609375f;    // float(log2 e)
  const float L_LO = 1.925963033500011079e-08f;     // log2 e - L_HI
  const float LN2 = 0.693147180559945309f;
  float th = -z * L_HI;
  float err = fmaf(-z, L_HI, -th);
  float tl = fmaf(-z, L_LO, err);
  th = fminf(th, 126.0f);
  float e = __builtin_amdgcn_exp2f(th);
  e = fmaf(e, tl * LN2, e);
  float d = 1.0f + e;
  float r = __builtin_amdgcn_rcpf(d);
  r = fmaf(r, fmaf(-d, r, 1.0f), r);
  e_out = e;
  return r;
}

__device__ __forceinline__ float sigmoid(float z) {
  float e;
  return sigmoid_e(z, e);
}

// sigma(z) and its slope sigma(z) (1 - sigma(z)) = e^-z sigma(z)^2.  The
// second form keeps full relative precision where sigma is close to 1 (there
// 1 - sigma would cancel); for z < -87 it underflows to 0 instead of ~1e-38.
__device__ __forceinline__ float sigmoid_slope(float z, float &slope) {
  float e;
  const float a = sigmoid_e(z, e);
  slope = (e * a) * a;
  return a;
}

// The tanh hidden activation (a variant; the paper's neurons are sigmoid)
// and its slope 1 - tanh(z)^2.
__device__ __forceinline__ float tanh_slope(float z, float &slope) {
  const float a = tanhf(z);
  slope = 1.0f - a * a;
  return a;
}

// Hidden activation by kind (0: sigma, 1: tanh) and its slope.
__device__ __forceinline__ float hidden_act(int act, float z, float &slope) {
  return act == 1 ? tanh_slope(z, slope) : sigmoid_slope(z, slope);
}

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

// v plus lane (v) permuted by a DPP row pattern (a VALU op, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float add_dpp(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false);
  return v + __builtin_bit_cast(float, s);
}

// Sum over each row of 16 lanes: swap neighbours, swap pairs, mirror within
// 8, mirror within 16.  Every lane of the row ends with the same value
// (each step adds two equal-order partial sums), so the result is bitwise
// identical across the row and across runs.
__device__ __forceinline__ float sum16(float v) {
  v = add_dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v = add_dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v = add_dpp<0x141>(v);  // row_half_mirror
  v = add_dpp<0x140>(v);  // row_mirror
  return v;
}

}  // namespace mlpk

// Launch wrappers implemented in the .hip files and used by the host API.
namespace mlph {

// Rows of one pass of the generic backward kernels (bounds their workspace).
constexpr int64_t kBackwardChunk = 16384;

// Small-network trainer: one workgroup per net, all epochs in one launch.
// items == nullptr means a single net described by `one`.  threads is 128,
// 256 or 512 (waves split the rows), or kHiddenSplit: one wave per 16
// hidden units of the widest net (waves split the hidden layer; the paper's
// sigmoid network without momentum, others fall back to 128 threads).
// small_threads picks it from the net count and a hint.
constexpr int kHiddenSplit = 64;
size_t small_lds_bytes(int n_rows, int n_hidden, int n_in, int threads, bool momentum = false);
size_t small_launch_lds_bytes(int max_rows, int max_hidden, int n_in, int threads, bool momentum = false);
int small_threads(int n_nets, int hint);
// act: hidden activation (0 sigma, 1 tanh); vel != nullptr: heavy-ball
// momentum mu with the velocity vel[P] (packed, a single net only).
hipError_t launch_small_train(const mlp_batch_item *items, mlp_batch_item one, int n_nets,
                              int n_in, int n_out, int max_rows, int max_hidden, const float *X,
                              const float *T, float *theta, float *comp, int epochs,
                              float *loss_hist, int act, float mu, float *vel, int threads, hipStream_t s);

// Generic layer kernels (any sizes) for mlp_forward / mlp_backward / mlp_step.
hipError_t launch_forward(int64_t n, int D, int H, int K, const float *X, mlp_params p, float *A,
                          float *Y, int act, hipStream_t s);
hipError_t launch_backward(int64_t n, int64_t ws_rows, int D, int H, int K, const float *X,
                           const float *A, const float *Y, const float *dY, const float *T,
                           mlp_params p, mlp_params g, float *dX, float *loss, float *ws, int act,
                           hipStream_t s);
hipError_t launch_step(int D, int H, int K, mlp_params p, mlp_params g, float *comp, float lr, float mu,
                       float *vel, hipStream_t s);
hipError_t launch_predict(int64_t n, int D, int H, int K, const float *X, mlp_params p, float *Y,
                          int32_t *labels, const float *T, int32_t *correct, int act, hipStream_t s);
// One dense layer (several-hidden-layer networks) and a packed update.
hipError_t launch_dense_forward(int64_t n, int din, int dout, const float *X, const float *W, const float *b,
                                int act, float *Y, hipStream_t s);
hipError_t launch_dense_backward(int64_t n, int din, int dout, const float *X, const float *Y, const float *dY,
                                 const float *W, int act, float *gW, float *gb, float *dX, float *dZ,
                                 hipStream_t s);
hipError_t launch_update(int64_t P, float *theta, const float *g, float *comp, float lr, hipStream_t s);
hipError_t launch_mse_grad(int64_t n, int k, const float *Y, const float *T, float *dY, float *loss, hipStream_t s);
hipError_t launch_eval_batched(const mlp_batch_item *items_dev, int n_nets, int D, int K, const float *X,
                               const float *T, const float *theta, float *loss, int32_t *correct, hipStream_t s);
hipError_t launch_cv_select(const float *loss, const int32_t *group, int n_nets, int n_groups, float *group_mean,
                            int32_t *best, hipStream_t s);

}  // namespace mlph
