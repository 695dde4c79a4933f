// Small-network trainer: one 256-thread workgroup trains one network, full
// batch, for all epochs in a single launch (arxiv 1908.07847, section 2.2:
// feed forward, error, backpropagation, gradient-descent update, repeated
// for a number of epochs).
//
// Everything a net touches lives in LDS for the whole run: the rows X (with
// a constant-1 column appended so that b1 is the last column of W1), the
// one-hot targets, W1|b1, W2|b2, and per epoch the activations A (with a
// constant-1 column so that b2 is the last column of W2), the hidden deltas
// and the output deltas.  HBM is read once at the start and written once at
// the end.  Each epoch is two barrier-separated phases:
//
//   F (row-parallel):  two threads per row, each owning half of the hidden
//     units.  z1 = [x 1] . [W1 b1]^T, a = sigma(z1), partial z2 over the
//     thread's hidden units combined with its partner lane, y = sigma(z2),
//     delta2 = 2 (y - t) / (N K) . y (1 - y), delta1 = (delta2 W2) . a (1 - a)
//     with the pre-update W2; the row's squared error feeds the loss.
//   G (parameter-parallel): each thread owns a 4x4 tile of [W1 b1] or of
//     [W2 b2], sums its gradient over the rows in row order (so every run is
//     bitwise repeatable), and applies the update to the master copy it keeps
//     in registers, with an optional Kahan compensation term, then publishes
//     the new weights to LDS for the next epoch's phase F.
//
// Limits: N <= 128 rows, H <= 64, D <= 48, K <= 4 (so at most 256 tiles).
#include "mlp_device.hpp"

namespace mlpk {

constexpr int kSmallThreads = 256;

struct SmallLayout {
  int N, H, D, K, DP, HP, HS, H2;
  __host__ __device__ SmallLayout(int n, int h, int d, int k) : N(n), H(h), D(d), K(k) {
    DP = (d + 1 + 3) / 4 * 4;        // x columns + bias column, padded to float4
    HP = (h + 1 + 7) / 8 * 8;        // hidden units + bias column, split in two float4 halves
    HS = HP + 4;                     // LDS row stride of A / delta1 (breaks bank aliasing)
    H2 = HP / 2;
  }
  // float offsets of each LDS region (all multiples of 4)
  __host__ __device__ int xs() const { return 0; }
  __host__ __device__ int w1() const { return xs() + N * DP; }
  __host__ __device__ int w2() const { return w1() + H * DP; }
  __host__ __device__ int a() const { return w2() + 4 * HS; }
  __host__ __device__ int d1() const { return a() + N * HS; }
  __host__ __device__ int d2() const { return d1() + N * HS; }
  __host__ __device__ int ts() const { return d2() + N * 4; }
  __host__ __device__ int red() const { return ts() + N * 4; }
  __host__ __device__ int total() const { return red() + 8; }
};

template <int DPM>
__global__ __launch_bounds__(kSmallThreads) void k_small_train(
    const mlp_batch_item *__restrict__ items, mlp_batch_item one, int D, int K,
    const float *__restrict__ X, const float *__restrict__ T, float *__restrict__ theta,
    float *__restrict__ comp, int epochs, float *__restrict__ loss_hist) {
  constexpr int H2M = 36;  // max hidden units per thread in phase F ((64+1 -> 72)/2)
  const mlp_batch_item it = items ? items[blockIdx.x] : one;
  const int N = it.n_rows, H = it.n_hidden;
  const float lr = it.lr;
  const SmallLayout L(N, H, D, K);
  const int DP = L.DP, HS = L.HS, H2 = L.H2;
  const int tid = threadIdx.x;

  extern __shared__ float4 smem4[];
  float *sm = reinterpret_cast<float *>(smem4);
  float *Xs = sm + L.xs();
  float *W1s = sm + L.w1();
  float *W2s = sm + L.w2();
  float *As = sm + L.a();
  float *D1s = sm + L.d1();
  float *D2s = sm + L.d2();
  float *Ts = sm + L.ts();
  float *red = sm + L.red();

  const float *Xg = X + it.x_off * D;
  const float *Tg = T + it.x_off * K;
  float *P = theta + it.p_off;
  float *C = comp ? comp + it.p_off : nullptr;
  const bool compensated = C != nullptr;
  const int oB1 = H * D, oW2 = oB1 + H, oB2 = oW2 + K * H;

  // ---- stage rows, targets; clear W2s (its padding must read as zero)
  for (int i = tid; i < N * DP; i += kSmallThreads) {
    int r = i / DP, c = i - r * DP;
    Xs[i] = c < D ? Xg[(int64_t)r * D + c] : (c == D ? 1.0f : 0.0f);
  }
  for (int i = tid; i < N * 4; i += kSmallThreads) {
    int r = i >> 2, k = i & 3;
    Ts[i] = k < K ? Tg[(int64_t)r * K + k] : 0.0f;
  }
  for (int i = tid; i < 4 * HS; i += kSmallThreads) W2s[i] = 0.0f;
  __syncthreads();

  // ---- phase-G tile ownership (fixed for the whole run)
  const int nTD = DP / 4;
  const int nT1 = ((H + 3) / 4) * nTD;   // tiles of [W1 b1]: 4 hidden x 4 columns
  const int nT2 = (H + 1 + 3) / 4;       // tiles of [W2 b2]: 4 outputs x 4 hidden(+bias)
  const bool own1 = tid < nT1;
  const bool own2 = !own1 && tid < nT1 + nT2;
  int th = 0, td = 0, tj = 0;
  if (own1) { th = tid / nTD; td = tid - th * nTD; }
  if (own2) tj = tid - nT1;

  float w[16], cw[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) { w[q] = 0.0f; cw[q] = 0.0f; }
  if (own1) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int h = 4 * th + i, d = 4 * td + j;
        if (h < H && d <= D) {
          int o = d < D ? h * D + d : oB1 + h;
          w[i * 4 + j] = P[o];
          cw[i * 4 + j] = compensated ? C[o] : 0.0f;
        }
        if (h < H) W1s[h * DP + d] = w[i * 4 + j];
      }
  } else if (own2) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int k = i, h = 4 * tj + j;
        if (k < K && h <= H) {
          int o = h < H ? oW2 + k * H + h : oB2 + k;
          w[i * 4 + j] = P[o];
          cw[i * 4 + j] = compensated ? C[o] : 0.0f;
          W2s[k * HS + h] = w[i * 4 + j];
        }
      }
  }
  __syncthreads();

  // ---- phase-F row ownership: two threads per row
  const int r = tid >> 1, half = tid & 1;
  const bool row_on = r < N;
  float x[DPM];
#pragma unroll
  for (int c = 0; c < DPM; ++c) x[c] = (row_on && c < DP) ? Xs[r * DP + c] : 0.0f;
  const float dscale = 2.0f / (float)(N * K);
  const float inv_nk = 1.0f / (float)(N * K);
  const int h0 = half * H2;

  for (int e = 0; e < epochs; ++e) {
    // ============================ phase F
    float sq = 0.0f;
    if (row_on) {
      float a[H2M];
#pragma unroll
      for (int j = 0; j < H2M; ++j) {
        a[j] = 0.0f;
        if (j < H2) {
          const int h = h0 + j;
          if (h < H) {
            const float4 *wr = reinterpret_cast<const float4 *>(W1s + h * DP);
            float z = 0.0f;
#pragma unroll
            for (int c4 = 0; c4 < DPM / 4; ++c4) {
              if (c4 < DP / 4) {
                float4 wv = wr[c4];
                z += x[4 * c4 + 0] * wv.x;
                z += x[4 * c4 + 1] * wv.y;
                z += x[4 * c4 + 2] * wv.z;
                z += x[4 * c4 + 3] * wv.w;
              }
            }
            a[j] = sigmoid(z);
          } else if (h == H) {
            a[j] = 1.0f;  // bias column of the output layer
          }
        }
      }
      float z2[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float s = 0.0f;
        if (k < K) {
          const float *w2r = W2s + k * HS + h0;
#pragma unroll
          for (int j = 0; j < H2M; ++j)
            if (j < H2) s += a[j] * w2r[j];
        }
        z2[k] = s;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) z2[k] += __shfl_xor(z2[k], 1, kWave);
      float d2[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        d2[k] = 0.0f;
        if (k < K) {
          float y = sigmoid(z2[k]);
          float err = y - Ts[r * 4 + k];
          sq += err * err;
          d2[k] = dscale * err * y * (1.0f - y);
        }
      }
      if (half) sq = 0.0f;  // the row's error is counted once
      float *arow = As + r * HS + h0;
      float *drow = D1s + r * HS + h0;
#pragma unroll
      for (int j4 = 0; j4 < H2M / 4; ++j4) {
        if (j4 < H2 / 4) {
          float dv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int j = 4 * j4 + u, h = h0 + j;
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (k < K) s += d2[k] * W2s[k * HS + h];
            dv[u] = h < H ? s * a[j] * (1.0f - a[j]) : 0.0f;
          }
          reinterpret_cast<float4 *>(arow)[j4] = make_float4(a[4 * j4], a[4 * j4 + 1], a[4 * j4 + 2], a[4 * j4 + 3]);
          reinterpret_cast<float4 *>(drow)[j4] = make_float4(dv[0], dv[1], dv[2], dv[3]);
        }
      }
      if (!half) reinterpret_cast<float4 *>(D2s)[r] = make_float4(d2[0], d2[1], d2[2], d2[3]);
    }
    if (loss_hist) {
      sq = wave_sum(sq);
      if ((tid & (kWave - 1)) == 0) red[tid / kWave] = sq;
    }
    __syncthreads();

    // ============================ phase G
    if (loss_hist && tid == 0)
      loss_hist[(int64_t)blockIdx.x * epochs + e] = ((red[0] + red[1]) + (red[2] + red[3])) * inv_nk;
    if (own1) {
      float acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
      const float *dcol = D1s + 4 * th;
      const float *xcol = Xs + 4 * td;
      for (int n = 0; n < N; ++n) {
        float4 dv = *reinterpret_cast<const float4 *>(dcol + n * HS);
        float4 xv = *reinterpret_cast<const float4 *>(xcol + n * DP);
        float dd[4] = {dv.x, dv.y, dv.z, dv.w}, xx[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i * 4 + j] += dd[i] * xx[j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int h = 4 * th + i, d = 4 * td + j;
          if (h < H && d <= D) {
            gd_update(w[i * 4 + j], cw[i * 4 + j], lr, acc[i * 4 + j], compensated);
            W1s[h * DP + d] = w[i * 4 + j];
          }
        }
    } else if (own2) {
      float acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
      const float *acol = As + 4 * tj;
      for (int n = 0; n < N; ++n) {
        float4 dv = reinterpret_cast<const float4 *>(D2s)[n];
        float4 av = *reinterpret_cast<const float4 *>(acol + n * HS);
        float dd[4] = {dv.x, dv.y, dv.z, dv.w}, aa[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i * 4 + j] += dd[i] * aa[j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int k = i, h = 4 * tj + j;
          if (k < K && h <= H) {
            gd_update(w[i * 4 + j], cw[i * 4 + j], lr, acc[i * 4 + j], compensated);
            W2s[k * HS + h] = w[i * 4 + j];
          }
        }
    }
    __syncthreads();
  }

  // ---- write the trained parameters (and compensation) back once
  if (own1) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int h = 4 * th + i, d = 4 * td + j;
        if (h < H && d <= D) {
          int o = d < D ? h * D + d : oB1 + h;
          P[o] = w[i * 4 + j];
          if (compensated) C[o] = cw[i * 4 + j];
        }
      }
  } else if (own2) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int k = i, h = 4 * tj + j;
        if (k < K && h <= H) {
          int o = h < H ? oW2 + k * H + h : oB2 + k;
          P[o] = w[i * 4 + j];
          if (compensated) C[o] = cw[i * 4 + j];
        }
      }
  }
}

}  // namespace mlpk

namespace mlph {

size_t small_lds_bytes(int n_rows, int n_hidden, int n_in) {
  mlpk::SmallLayout L(n_rows, n_hidden, n_in, 4);
  return sizeof(float) * (size_t)L.total();
}

hipError_t launch_small_train(const mlp_batch_item *items, mlp_batch_item one, int n_nets,
                              int n_in, int n_out, int max_rows, int max_hidden, const float *X,
                              const float *T, float *theta, float *comp, int epochs,
                              float *loss_hist, hipStream_t s) {
  size_t lds = small_lds_bytes(max_rows, max_hidden, n_in);
  dim3 grid(n_nets), block(mlpk::kSmallThreads);
  if (n_in + 1 <= 36) {
    auto kern = mlpk::k_small_train<36>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, block, lds, s, items, one, n_in, n_out, X, T, theta, comp,
                       epochs, loss_hist);
  } else {
    auto kern = mlpk::k_small_train<52>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, block, lds, s, items, one, n_in, n_out, X, T, theta, comp,
                       epochs, loss_hist);
  }
  return hipGetLastError();
}

}  // namespace mlph
