// One fully connected layer and its adjoint: the building block of networks
// with several hidden layers (section 2.2's layer, stacked; the paper's
// network has one hidden layer).
//
//   k_dense_fwd<ACT>  Y = act(X W^T + b); a workgroup computes 64 rows x 64
//                     outputs, 16 rows per wave, on v_mfma_f32_16x16x4_f32
//                     with X and W staged in LDS in chunks of 32 inputs
//   k_dense_dz<ACT>   dZ = dY . act'(Y)   (act' from the layer's output)
//   k_dense_wsum      gW[o][i] = sum_r dZ[r][o] X[r][i], gb[o] = sum_r dZ[r][o]:
//                     one wave per parameter, lanes over rows, fixed butterfly
//                     (bitwise repeatable)
//   k_dense_dx        dX[r][i] = sum_o dZ[r][o] W[o][i], one thread per entry
//   k_update          theta <- theta - lr g over a packed parameter vector,
//                     optionally Kahan-compensated
//   k_mse_grad        the error of section 2.2 read as the mean squared error,
//                     L = sum (Y-T)^2 / (n K), and dL/dY = 2 (Y-T) / (n K); one
//                     workgroup, threads strided over the entries, a fixed-order
//                     block sum (bitwise repeatable)
// ACT: 0 the sigmoid of Equation 1, 1 tanh.
#include "mlp_device.hpp"

namespace mlpk {

constexpr int kDR = 64, kDO = 64, kDK = 32;

typedef float f32x4_d __attribute__((ext_vector_type(4)));

template <int ACT>
__device__ __forceinline__ float dense_act(float z) {
  float slope;
  return hidden_act(ACT, z, slope);
}

template <int ACT>
__global__ __launch_bounds__(256) void k_dense_fwd(int64_t n, int din, int dout, const float *__restrict__ X,
                                                   const float *__restrict__ W, const float *__restrict__ b,
                                                   float *__restrict__ Y) {
  __shared__ float xs[kDR][kDK + 1];
  __shared__ float ws[kDO][kDK + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, lg = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kDR;
  const int o0 = blockIdx.y * kDO;
  f32x4_d acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4_d{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < din; k0 += kDK) {
    __syncthreads();   // the previous chunk is no longer read
    for (int q = tid; q < kDR * kDK; q += 256) {
      const int r = q / kDK, c = q - r * kDK;
      xs[r][c] = (r0 + r < n && k0 + c < din) ? X[(r0 + r) * din + k0 + c] : 0.0f;
    }
    for (int q = tid; q < kDO * kDK; q += 256) {
      const int o = q / kDK, c = q - o * kDK;
      ws[o][c] = (o0 + o < dout && k0 + c < din) ? W[(int64_t)(o0 + o) * din + k0 + c] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kDK; kk += 4) {
      const float a = xs[wave * 16 + l16][kk + lg];   // A: rows x inputs
#pragma unroll
      for (int t = 0; t < 4; ++t)                     // B: inputs x outputs
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, ws[t * 16 + l16][kk + lg], acc[t], 0, 0, 0);
    }
  }
  // lane (output l16 of tile t, group lg) holds rows 4 lg .. 4 lg + 3 of the wave's 16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int o = o0 + t * 16 + l16;
    if (o >= dout) continue;
    const float bo = b[o];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = r0 + wave * 16 + 4 * lg + i;
      if (r < n) Y[r * dout + o] = dense_act<ACT>(acc[t][i] + bo);
    }
  }
}

template <int ACT>
__global__ __launch_bounds__(256) void k_dense_dz(int64_t m, const float *__restrict__ Y, const float *__restrict__ dY,
                                                  float *__restrict__ dZ) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const float y = Y[q];
  dZ[q] = dY[q] * (ACT == 1 ? 1.0f - y * y : y * (1.0f - y));
}

__global__ __launch_bounds__(256) void k_dense_wsum(int64_t n, int din, int dout, const float *__restrict__ X,
                                                    const float *__restrict__ dZ, float *__restrict__ gW,
                                                    float *__restrict__ gb) {
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nw = (int64_t)dout * din;
  if (q >= nw + dout) return;   // whole waves leave together
  float s = 0.0f;
  if (q < nw) {
    const int o = (int)(q / din), i = (int)(q - (int64_t)o * din);
    for (int64_t r = lane; r < n; r += kWave) s = fmaf(dZ[r * dout + o], X[r * din + i], s);
    s = wave_sum(s);
    if (lane == 0) gW[q] = s;
  } else {
    const int o = (int)(q - nw);
    for (int64_t r = lane; r < n; r += kWave) s += dZ[r * dout + o];
    s = wave_sum(s);
    if (lane == 0) gb[o] = s;
  }
}

__global__ __launch_bounds__(256) void k_dense_dx(int64_t n, int din, int dout, const float *__restrict__ dZ,
                                                  const float *__restrict__ W, float *__restrict__ dX) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * din) return;
  const int64_t r = q / din;
  const int i = (int)(q - r * din);
  float s = 0.0f;
  for (int o = 0; o < dout; ++o) s = fmaf(dZ[r * dout + o], W[(int64_t)o * din + i], s);
  dX[q] = s;
}

__global__ __launch_bounds__(256) void k_update(int64_t P, float *__restrict__ theta, const float *__restrict__ g,
                                                float *__restrict__ comp, float lr) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  float w = theta[q], c = comp ? comp[q] : 0.0f;
  gd_update(w, c, lr, g[q], comp != nullptr);
  theta[q] = w;
  if (comp) comp[q] = c;
}

__global__ __launch_bounds__(1024) void k_mse_grad(int64_t m, float scale, const float *__restrict__ Y,
                                                   const float *__restrict__ T, float *__restrict__ dY,
                                                   float *__restrict__ loss) {
  __shared__ float part[16];
  float s = 0.0f;
  for (int64_t q = threadIdx.x; q < m; q += blockDim.x) {
    const float e = Y[q] - T[q];
    s = fmaf(e, e, s);
    dY[q] = 2.0f * e * scale;
  }
  s = wave_sum(s);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += part[w];
    if (loss) loss[0] = t * scale;
  }
}

}  // namespace mlpk

namespace mlph {

static dim3 blocks_for(int64_t n, int per) { return dim3((unsigned)((n + per - 1) / per)); }

hipError_t launch_dense_forward(int64_t n, int din, int dout, const float *X, const float *W, const float *b,
                                int act, float *Y, hipStream_t s) {
  const dim3 grid((unsigned)((n + mlpk::kDR - 1) / mlpk::kDR), (unsigned)((dout + mlpk::kDO - 1) / mlpk::kDO));
  if (act == 1)
    hipLaunchKernelGGL(mlpk::k_dense_fwd<1>, grid, dim3(256), 0, s, n, din, dout, X, W, b, Y);
  else
    hipLaunchKernelGGL(mlpk::k_dense_fwd<0>, grid, dim3(256), 0, s, n, din, dout, X, W, b, Y);
  return hipGetLastError();
}

hipError_t launch_dense_backward(int64_t n, int din, int dout, const float *X, const float *Y, const float *dY,
                                 const float *W, int act, float *gW, float *gb, float *dX, float *dZ,
                                 hipStream_t s) {
  const int64_t m = n * dout;
  if (act == 1)
    hipLaunchKernelGGL(mlpk::k_dense_dz<1>, blocks_for(m, 256), dim3(256), 0, s, m, Y, dY, dZ);
  else
    hipLaunchKernelGGL(mlpk::k_dense_dz<0>, blocks_for(m, 256), dim3(256), 0, s, m, Y, dY, dZ);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlpk::k_dense_wsum, blocks_for((int64_t)dout * din + dout, 256 / mlpk::kWave), dim3(256), 0, s,
                     n, din, dout, X, dZ, gW, gb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (dX) {
    hipLaunchKernelGGL(mlpk::k_dense_dx, blocks_for(n * din, 256), dim3(256), 0, s, n, din, dout, dZ, W, dX);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_mse_grad(int64_t n, int k, const float *Y, const float *T, float *dY, float *loss, hipStream_t s) {
  const int64_t m = n * k;
  hipLaunchKernelGGL(mlpk::k_mse_grad, dim3(1), dim3(1024), 0, s, m, 1.0f / ((float)n * (float)k), Y, T, dY, loss);
  return hipGetLastError();
}

hipError_t launch_update(int64_t P, float *theta, const float *g, float *comp, float lr, hipStream_t s) {
  hipLaunchKernelGGL(mlpk::k_update, blocks_for(P, 256), dim3(256), 0, s, P, theta, g, comp, lr);
  return hipGetLastError();
}

}  // namespace mlph
