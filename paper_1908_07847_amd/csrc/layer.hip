// Separate forward / backward / update kernels (arxiv 1908.07847,
// section 2.2), for callers that drive the steps themselves -- e.g. a
// torch.autograd.Function whose backward is this hand-written adjoint.
//
//  k_forward_tiled 64 rows per workgroup, 16 per wave: the row tile of X and
//                  a 64-unit block of W1 at a time in LDS, z1 on
//                  v_mfma_f32_16x16x4_f32, sigma in the accumulator layout,
//                  the output layer as lane partials summed across the 16
//                  lanes of a row (n_in <= 256, n_out <= 16)
//  k_forward       one thread per row (any n_in): z1 = X W1^T + b1,
//                  A = sigma(z1), Y = sigma(A W2^T + b2).
//  k_backward_rows one thread per row: delta2 = dY . Y (1 - Y) (dY from the
//                  caller, or the MSE reading 2 (Y - T) / (n K)),
//                  delta1 = (delta2 W2) . A (1 - A); optional dX = delta1 W1;
//                  writes delta1, delta2 and the row's squared error.
//  k_backward_sum  one wave per parameter (plus one for the loss): lane
//                  partial sums over the rows, then a fixed butterfly, so
//                  the result is bitwise repeatable.
//  k_step          theta <- theta - lr g, optionally Kahan-compensated; with
//                  a velocity buffer, heavy-ball momentum (v <- mu v + g,
//                  theta <- theta - lr v).  Forward and backward take the
//                  hidden activation (sigma, or the tanh variant).
//  k_eval_batched  one workgroup per net of a batched item table: loss and
//                  correct count of the net on its own rows (e.g. a held-out
//                  fold), threads over rows, fixed-order block sums
//  k_argmax        rows in a grid-stride loop (at most 512 workgroups): the
//                  class is the index of the largest
//                  output (lowest index on ties); with one-hot targets, the
//                  count of rows whose class matches the target's, summed
//                  per block and added once per block (integer adds, so the
//                  count does not depend on their order).
#include <algorithm>

#include "mlp_device.hpp"

namespace mlpk {

__global__ __launch_bounds__(256) void k_forward(int64_t n, int D, int H, int K,
                                                 const float *__restrict__ X, mlp_params p,
                                                 float *__restrict__ A, float *__restrict__ Y, int act) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float *x = X + r * D;
  float z2[kLayerMaxOut];
  for (int k = 0; k < K && k < kLayerMaxOut; ++k) z2[k] = p.b2[k];
  for (int h = 0; h < H; ++h) {
    const float *w = p.W1 + (int64_t)h * D;
    float z = p.b1[h];
    for (int d = 0; d < D; ++d) z += x[d] * w[d];
    float slope;
    const float a = hidden_act(act, z, slope);
    if (A) A[r * H + h] = a;
    for (int k = 0; k < K && k < kLayerMaxOut; ++k) z2[k] += a * p.W2[(int64_t)k * H + h];
  }
  for (int k = 0; k < K && k < kLayerMaxOut; ++k) Y[r * K + k] = sigmoid(z2[k]);
}

constexpr int kFwdRows = 64, kFwdHB = 64, kFwdMaxD = 256;

typedef float f32x4_l __attribute__((ext_vector_type(4)));

// KO: output slots held per row in registers (K <= KO); ACT: the hidden
// activation (0 sigma, 1 tanh).
template <int KO, int ACT>
__global__ __launch_bounds__(256) void k_forward_tiled(int64_t n, int D, int H, int K,
                                                       const float *__restrict__ X, mlp_params p,
                                                       float *__restrict__ A, float *__restrict__ Y) {
  extern __shared__ float4 fsm4[];
  float *sm = reinterpret_cast<float *>(fsm4);
  const int DK = (D + 3) / 4 * 4, XS = DK + 1;     // contraction length; odd row stride
  float *xs = sm;                                   // [64][XS]
  float *ws = xs + kFwdRows * XS;                   // [64][XS] W1 block
  float *w2 = ws + kFwdHB * XS;                     // [16][64] W2 block
  float *b1 = w2 + kLayerMaxOut * kFwdHB;           // [64]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kFwdRows;
  const int rows = (int)min((int64_t)kFwdRows, n - r0);
  for (int q = tid; q < kFwdRows * XS; q += 256) {
    const int r = q / XS, c = q - r * XS;
    xs[q] = (r < rows && c < D) ? X[(r0 + r) * D + c] : 0.0f;
  }
  float zp[4][KO];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < KO; ++k) zp[i][k] = 0.0f;
  for (int h0 = 0; h0 < H; h0 += kFwdHB) {
    __syncthreads();   // the previous block's W1 / W2 are no longer read
    for (int q = tid; q < kFwdHB * XS; q += 256) {
      const int h = q / XS, c = q - h * XS;
      ws[q] = (h0 + h < H && c < D) ? p.W1[(int64_t)(h0 + h) * D + c] : 0.0f;
    }
    for (int q = tid; q < kLayerMaxOut * kFwdHB; q += 256) {
      const int k = q / kFwdHB, h = q - k * kFwdHB;
      w2[q] = (k < K && h0 + h < H) ? p.W2[(int64_t)k * H + h0 + h] : 0.0f;
    }
    if (tid < kFwdHB) b1[tid] = h0 + tid < H ? p.b1[h0 + tid] : 0.0f;
    __syncthreads();
    for (int ht = 0; ht < kFwdHB / 16; ++ht) {
      if (h0 + ht * 16 >= H) break;
      f32x4_l z = {0.f, 0.f, 0.f, 0.f};
      const float *xa = xs + (wave * 16 + l16) * XS + lg;
      const float *wb = ws + (ht * 16 + l16) * XS + lg;
      for (int k0 = 0; k0 < DK; k0 += 4) z = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[k0], wb[k0], z, 0, 0, 0);
      const int hl = ht * 16 + l16, h = h0 + hl;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wave * 16 + 4 * lg + i;
        float slope;
        const float a = h < H ? hidden_act(ACT, z[i] + b1[hl], slope) : 0.0f;
        if (A && r < rows && h < H) A[(r0 + r) * H + h] = a;
#pragma unroll
        for (int k = 0; k < KO; ++k)
          if (k < K) zp[i][k] = fmaf(a, w2[k * kFwdHB + hl], zp[i][k]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = wave * 16 + 4 * lg + i;
#pragma unroll
    for (int k = 0; k < KO; ++k) {
      if (k < K) {
        const float z2 = sum16(zp[i][k]);
        if (l16 == 0 && r < rows) Y[(r0 + r) * K + k] = sigmoid(z2 + p.b2[k]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_backward_rows(
    int64_t n, int64_t n_total, int D, int H, int K, const float *__restrict__ A, const float *__restrict__ Y,
    const float *__restrict__ dY, const float *__restrict__ T, mlp_params p,
    float *__restrict__ dX, float *__restrict__ d1_out, float *__restrict__ d2_out,
    float *__restrict__ sq_out, int act) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float mse_scale = 2.0f / ((float)n_total * (float)K);
  float sq = 0.0f;
  for (int k = 0; k < K; ++k) {
    float y = Y[r * K + k];
    float g;
    if (dY) {
      g = dY[r * K + k];
    } else {
      float err = y - T[r * K + k];
      sq += err * err;
      g = mse_scale * err;
    }
    d2_out[r * K + k] = g * y * (1.0f - y);
  }
  sq_out[r] = sq;
  for (int h = 0; h < H; ++h) {
    float s = 0.0f;
    for (int k = 0; k < K; ++k) s += d2_out[r * K + k] * p.W2[(int64_t)k * H + h];
    float a = A[r * H + h];
    d1_out[r * H + h] = act == 1 ? s * (1.0f - a * a) : s * a * (1.0f - a);
  }
  if (dX) {
    for (int d = 0; d < D; ++d) {
      float s = 0.0f;
      for (int h = 0; h < H; ++h) s += d1_out[r * H + h] * p.W1[(int64_t)h * D + d];
      dX[r * D + d] = s;
    }
  }
}

// One wave per parameter q in packed order [W1 | b1 | W2 | b2], plus q == P
// for the loss: lane l sums rows l, l + 64, ... in order, then a fixed
// butterfly adds the 64 lane sums, so the result is bitwise repeatable.
__global__ __launch_bounds__(256) void k_backward_sum(
    int64_t n, int64_t n_total, int accumulate, int D, int H, int K, const float *__restrict__ X,
    const float *__restrict__ A, const float *__restrict__ d1, const float *__restrict__ d2,
    const float *__restrict__ sq, mlp_params g, float *__restrict__ loss) {
  const int64_t P = (int64_t)D * H + H + (int64_t)H * K + K;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  if (q > P) return;   // whole waves leave together
  float s = 0.0f;
  if (q < (int64_t)D * H) {
    const int h = (int)(q / D), d = (int)(q - (int64_t)h * D);
    for (int64_t r = lane; r < n; r += kWave) s += d1[r * H + h] * X[r * D + d];
    s = wave_sum(s);
    if (lane == 0) g.W1[q] = accumulate ? g.W1[q] + s : s;
  } else if (q < (int64_t)D * H + H) {
    const int h = (int)(q - (int64_t)D * H);
    for (int64_t r = lane; r < n; r += kWave) s += d1[r * H + h];
    s = wave_sum(s);
    if (lane == 0) g.b1[h] = accumulate ? g.b1[h] + s : s;
  } else if (q < (int64_t)D * H + H + (int64_t)H * K) {
    const int64_t o = q - ((int64_t)D * H + H);
    const int k = (int)(o / H), h = (int)(o - (int64_t)k * H);
    for (int64_t r = lane; r < n; r += kWave) s += d2[r * K + k] * A[r * H + h];
    s = wave_sum(s);
    if (lane == 0) g.W2[o] = accumulate ? g.W2[o] + s : s;
  } else if (q < P) {
    const int k = (int)(q - ((int64_t)D * H + H + (int64_t)H * K));
    for (int64_t r = lane; r < n; r += kWave) s += d2[r * K + k];
    s = wave_sum(s);
    if (lane == 0) g.b2[k] = accumulate ? g.b2[k] + s : s;
  } else if (loss) {
    for (int64_t r = lane; r < n; r += kWave) s += sq[r];
    s = wave_sum(s) / ((float)n_total * (float)K);
    if (lane == 0) loss[0] = accumulate ? loss[0] + s : s;
  }
}

__global__ __launch_bounds__(256) void k_step(int D, int H, int K, mlp_params p, mlp_params g,
                                              float *__restrict__ comp, float lr, float mu,
                                              float *__restrict__ vel) {
  const int64_t P = (int64_t)D * H + H + (int64_t)H * K + K;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  float *w;
  const float *gr;
  const int64_t oB1 = (int64_t)D * H, oW2 = oB1 + H, oB2 = oW2 + (int64_t)H * K;
  if (q < oB1) { w = p.W1 + q; gr = g.W1 + q; }
  else if (q < oW2) { w = p.b1 + (q - oB1); gr = g.b1 + (q - oB1); }
  else if (q < oB2) { w = p.W2 + (q - oW2); gr = g.W2 + (q - oW2); }
  else { w = p.b2 + (q - oB2); gr = g.b2 + (q - oB2); }
  float wv = *w, c = comp ? comp[q] : 0.0f;
  float step = *gr;
  if (vel) {   // heavy-ball momentum: v <- mu v + g, theta <- theta - lr v
    step = fmaf(mu, vel[q], step);
    vel[q] = step;
  }
  gd_update(wv, c, lr, step, comp != nullptr);
  *w = wv;
  if (comp) comp[q] = c;
}

}  // namespace mlpk

namespace mlpk {

__global__ void k_fill_i32(int32_t *p, int32_t v) { *p = v; }

// Class of a row of outputs (or targets): the largest entry, the lowest
// index on ties; a single output is a two-class net, class 1 above 1/2.
__device__ __forceinline__ int argmax_row(const float *v, int K) {
  if (K == 1) return v[0] > 0.5f ? 1 : 0;
  int best = 0;
  for (int k = 1; k < K; ++k)
    if (v[k] > v[best]) best = k;   // strict: the lowest index wins ties
  return best;
}

__global__ __launch_bounds__(256) void k_eval_batched(const mlp_batch_item *__restrict__ items, int D, int K,
                                                      const float *__restrict__ X, const float *__restrict__ T,
                                                      const float *__restrict__ theta, float *__restrict__ loss,
                                                      int32_t *__restrict__ correct) {
  const mlp_batch_item it = items[blockIdx.x];
  const int N = it.n_rows, H = it.n_hidden;
  const float *W1 = theta + it.p_off, *b1 = W1 + (int64_t)H * D, *W2 = b1 + H, *b2 = W2 + (int64_t)K * H;
  float sq = 0.0f;
  int hit = 0;
  for (int r = threadIdx.x; r < N; r += blockDim.x) {
    const float *x = X + (it.x_off + r) * D;
    const float *t = T + (it.x_off + r) * K;
    float z2[MLP_SMALL_MAX_OUT];
#pragma unroll
    for (int k = 0; k < MLP_SMALL_MAX_OUT; ++k) z2[k] = k < K ? b2[k] : 0.0f;
    for (int h = 0; h < H; ++h) {
      const float *w = W1 + (int64_t)h * D;
      float z = b1[h];
      for (int d = 0; d < D; ++d) z = fmaf(x[d], w[d], z);
      const float a = sigmoid(z);
#pragma unroll
      for (int k = 0; k < MLP_SMALL_MAX_OUT; ++k)
        if (k < K) z2[k] = fmaf(a, W2[(int64_t)k * H + h], z2[k]);
    }
    float y[MLP_SMALL_MAX_OUT];
#pragma unroll
    for (int k = 0; k < MLP_SMALL_MAX_OUT; ++k) {
      y[k] = sigmoid(z2[k]);
      if (k < K) {
        const float e = y[k] - t[k];
        sq = fmaf(e, e, sq);
      }
    }
    hit += argmax_row(y, K) == argmax_row(t, K);
  }
  __shared__ float ps[4];
  __shared__ int ph[4];
  float v = wave_sum(sq);
  int c = hit;
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, kWave);
  if ((threadIdx.x & 63) == 0) {
    ps[threadIdx.x >> 6] = v;
    ph[threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    loss[blockIdx.x] = ((ps[0] + ps[1]) + (ps[2] + ps[3])) / ((float)N * (float)K);
    if (correct) correct[blockIdx.x] = (ph[0] + ph[1]) + (ph[2] + ph[3]);
  }
}

__global__ __launch_bounds__(256) void k_argmax(int64_t n, int K, const float *__restrict__ Y,
                                                const float *__restrict__ T, int32_t *__restrict__ labels,
                                                int32_t *__restrict__ correct) {
  int hit = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int c = argmax_row(Y + r * K, K);
    labels[r] = c;
    if (T) hit += c == argmax_row(T + r * K, K);
  }
  if (T) {
    __shared__ int part[4];
    int v = hit;
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(correct, (part[0] + part[1]) + (part[2] + part[3]));
  }
}

}  // namespace mlpk

namespace mlph {

static dim3 grid_for(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

hipError_t launch_forward(int64_t n, int D, int H, int K, const float *X, mlp_params p, float *A,
                          float *Y, int act, hipStream_t s) {
  if (D <= mlpk::kFwdMaxD && K <= mlpk::kLayerMaxOut) {
    const int XS = (D + 3) / 4 * 4 + 1;
    const size_t lds = sizeof(float) * ((size_t)(mlpk::kFwdRows + mlpk::kFwdHB) * XS +
                                        mlpk::kLayerMaxOut * mlpk::kFwdHB + mlpk::kFwdHB);
    using mlpk::k_forward_tiled;
    using mlpk::kLayerMaxOut;
    const void *kern = K <= 4 ? (act ? (const void *)k_forward_tiled<4, 1> : (const void *)k_forward_tiled<4, 0>)
                              : (act ? (const void *)k_forward_tiled<kLayerMaxOut, 1>
                                     : (const void *)k_forward_tiled<kLayerMaxOut, 0>);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int64_t blocks = (n + mlpk::kFwdRows - 1) / mlpk::kFwdRows;
    void *args[] = {&n, &D, &H, &K, &X, &p, &A, &Y};
    e = hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(256), args, lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  hipLaunchKernelGGL(mlpk::k_forward, grid_for(n, 256), dim3(256), 0, s, n, D, H, K, X, p, A, Y, act);
  return hipGetLastError();
}

}  // namespace mlph

namespace mlpk {

// Cross-validation selection: one workgroup.  Thread t owns the groups t,
// t + 1024, ...: for each it walks every net in increasing order (the
// (loss, group) pairs staged through LDS in chunks, read as broadcasts), so a
// mean is one fixed-order float32 sum.  Then a (mean, group) minimum over
// the threads, ties to the lower group.
constexpr int kSelThreads = 1024;
constexpr int kSelChunk = 2048;
__global__ __launch_bounds__(kSelThreads) void k_cv_select(const float *__restrict__ loss,
                                                         const int32_t *__restrict__ group, int n, int ng,
                                                         float *__restrict__ mean, int32_t *__restrict__ best) {
  __shared__ float ls[kSelChunk];
  __shared__ int32_t gs[kSelChunk];
  __shared__ float bv[kSelThreads];
  __shared__ int32_t bi[kSelThreads];
  const int t = threadIdx.x;
  float mv = __builtin_inff();
  int mi = 0x7fffffff;
  for (int r = 0; r * kSelThreads < ng; ++r) {
    const int g = t + r * kSelThreads;
    float sum = 0.0f;
    int cnt = 0;
    for (int c0 = 0; c0 < n; c0 += kSelChunk) {
      const int m = min(kSelChunk, n - c0);
      __syncthreads();   // the previous chunk is no longer read
      for (int i = t; i < m; i += kSelThreads) {
        ls[i] = loss[c0 + i];
        gs[i] = group[c0 + i];
      }
      __syncthreads();
      if (g < ng)
        for (int i = 0; i < m; ++i)
          if (gs[i] == g) {
            sum += ls[i];
            cnt += 1;
          }
    }
    if (g < ng) {
      float v = cnt ? sum / (float)cnt : __builtin_inff();
      if (!(v < __builtin_inff())) v = __builtin_inff();   // NaN or +inf
      mean[g] = v;
      if (v < mv || (v == mv && g < mi)) {
        mv = v;
        mi = g;
      }
    }
  }
  bv[t] = mv;
  bi[t] = mi;
  __syncthreads();
  for (int st = kSelThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      const float v = bv[t + st];
      const int i = bi[t + st];
      if (v < bv[t] || (v == bv[t] && i < bi[t])) {
        bv[t] = v;
        bi[t] = i;
      }
    }
    __syncthreads();
  }
  if (t == 0) best[0] = bi[0] == 0x7fffffff ? 0 : bi[0];
}

}  // namespace mlpk

namespace mlph {

hipError_t launch_cv_select(const float *loss, const int32_t *group, int n_nets, int n_groups, float *group_mean,
                            int32_t *best, hipStream_t s) {
  hipLaunchKernelGGL(mlpk::k_cv_select, dim3(1), dim3(mlpk::kSelThreads), 0, s, loss, group, n_nets, n_groups,
                     group_mean, best);
  return hipGetLastError();
}

hipError_t launch_eval_batched(const mlp_batch_item *items_dev, int n_nets, int D, int K, const float *X,
                               const float *T, const float *theta, float *loss, int32_t *correct, hipStream_t s) {
  hipLaunchKernelGGL(mlpk::k_eval_batched, dim3(n_nets), dim3(256), 0, s, items_dev, D, K, X, T, theta, loss,
                     correct);
  return hipGetLastError();
}

hipError_t launch_predict(int64_t n, int D, int H, int K, const float *X, mlp_params p, float *Y,
                          int32_t *labels, const float *T, int32_t *correct, int act, hipStream_t s) {
  hipError_t e = launch_forward(n, D, H, K, X, p, nullptr, Y, act, s);
  if (e != hipSuccess) return e;
  if (T) {
    hipLaunchKernelGGL(mlpk::k_fill_i32, dim3(1), dim3(1), 0, s, correct, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // at most 512 blocks (rows in a grid-stride loop): one count add per block
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(512, (n + 255) / 256)));
  hipLaunchKernelGGL(mlpk::k_argmax, grid, dim3(256), 0, s, n, K, Y, T, labels, correct);
  return hipGetLastError();
}

// ws layout (floats): delta1 [chunk][H] | delta2 [chunk][K] | sq [chunk].  Rows
// are processed in chunks of at most ws_rows; each chunk's sums are
// added to the previous ones in chunk order (fixed, so still repeatable).
hipError_t launch_backward(int64_t n, int64_t ws_rows, int D, int H, int K, const float *X,
                           const float *A, const float *Y, const float *dY, const float *T,
                           mlp_params p, mlp_params g, float *dX, float *loss, float *ws, int act,
                           hipStream_t s) {
  const int64_t chunk = std::min<int64_t>(n, ws_rows);
  float *d1 = ws, *d2 = ws + chunk * H, *sq = d2 + chunk * K;
  const int64_t P = (int64_t)D * H + H + (int64_t)H * K + K;
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int64_t m = std::min(chunk, n - r0);
    hipLaunchKernelGGL(mlpk::k_backward_rows, grid_for(m, 256), dim3(256), 0, s, m, n, D, H, K,
                       A + r0 * H, Y + r0 * K, dY ? dY + r0 * K : nullptr, T ? T + r0 * K : nullptr,
                       p, dX ? dX + r0 * D : nullptr, d1, d2, sq, act);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlpk::k_backward_sum, grid_for(P + 1, 256 / mlpk::kWave), dim3(256), 0, s, m, n,
                       r0 > 0 ? 1 : 0, D, H, K, X + r0 * D, A + r0 * H, d1, d2, sq, g,
                       dY ? nullptr : loss);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_step(int D, int H, int K, mlp_params p, mlp_params g, float *comp, float lr, float mu,
                       float *vel, hipStream_t s) {
  const int64_t P = (int64_t)D * H + H + (int64_t)H * K + K;
  hipLaunchKernelGGL(mlpk::k_step, grid_for(P, 256), dim3(256), 0, s, D, H, K, p, g, comp, lr, mu, vel);
  return hipGetLastError();
}

}  // namespace mlph
