// Fused trainer for networks with several hidden layers (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mlph {

constexpr int kDeepMaxLayers = 8;      // weight layers
constexpr int kDeepMaxWidth = 1024;    // units of any layer
constexpr int kDeepThreads = 1024;

// LDS plan of one network (floats).  Row strides are odd so that the lanes
// of a wave walking rows of an activation or delta array hit distinct banks,
// and leave room after each row of a layer's input for a column of ones
// (the bias input of the gradient's row sums).
struct DeepPlan {
  int L, n, P, RS, seg;            // layers, rows, parameters, row segments of the gradient sums
  int w[kDeepMaxLayers + 1];       // widths
  int sa[kDeepMaxLayers + 1];      // row stride of layer l's activations (l = 0: X), >= w[l] + 1
  int poff[kDeepMaxLayers + 1];    // packed offset of W_l (b_l follows it); poff[L] = P
  int aoff[kDeepMaxLayers + 1];    // LDS offset of layer l's activations
  int toff, d0, d1, sd;            // targets, the two delta buffers and their row stride
  int th, cp, gr, red;             // parameters, compensation, RS gradient copies, reduction slots
  int total;                       // floats of LDS
};

// Plans the LDS layout; false when the network does not fit in `lds_max`
// bytes (or a width or the layer count is out of range).
bool deep_plan(int L, const int32_t *widths, int64_t n, size_t lds_max, DeepPlan *p);

hipError_t launch_deep_train(const DeepPlan &p, int act, const float *X, const float *T, float *theta,
                             float *comp, float lr, int epochs, float *loss_hist, hipStream_t s);

}  // namespace mlph
