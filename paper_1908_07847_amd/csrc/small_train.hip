// Small-network trainer: one workgroup trains one network, full batch, for
// all epochs in a single launch (arxiv 1908.07847, section 2.2: feed
// forward, error, backpropagation, gradient-descent update, repeated for a
// number of epochs).
//
// Everything a net touches lives in LDS for the whole run: its rows X (with
// a constant-1 column appended, so b1 is the last column of W1), the one-hot
// targets, W1|b1, W2|b2, and per epoch the activations A (with a constant-1
// column, so b2 is the last column of W2), the hidden deltas and the output
// deltas.  HBM is read once at the start and written once at the end.
// Each epoch is two barrier-separated phases:
//
//   F (row-parallel): S threads per row, each owning a contiguous slice of
//     the hidden units.  z1 = [x 1].[W1 b1]^T, a = sigma(z1), partial
//     z2 = a.[W2 b2]^T over the slice, summed across the row's S lanes,
//     y = sigma(z2), delta2 = 2 (y - t) / (N K) . y (1 - y),
//     delta1 = (delta2 W2) . a (1 - a) with the pre-update W2.
//   G (parameter-parallel): the gradient is cut into 4x4 tiles of [W1 b1]
//     and [W2 b2]; C adjacent lanes share a tile and each sums every C-th
//     row, then a fixed butterfly over those lanes adds the C partial sums
//     (bitwise repeatable).  The tile's first lane keeps the master weights
//     and their Kahan compensation in registers for the whole run, applies
//     the update and publishes the new weights to LDS.
//
// NT (threads per workgroup) is a template parameter: 1024 when one net has
// the chip to itself (its epoch latency is the whole story), 256 when many
// nets share the CUs (several workgroups per CU hide each other's latency).
// Limits: N <= 128 rows, H <= 64, D <= 48, K <= 4.
#include <algorithm>

#include "mlp_device.hpp"

namespace mlpk {

struct SmallLayout {
  int N, H, D, K, DP, HA, HP4, S, HPT, HR, HS;
  __host__ __device__ SmallLayout(int n, int h, int d, int k, int nt) : N(n), H(h), D(d), K(k) {
    DP = (d + 1 + 3) / 4 * 4;         // features + bias column, float4 padded
    HA = h + 1;                       // hidden units + bias column
    HP4 = (HA + 3) / 4 * 4;
    S = 1;                            // threads per row in phase F
    while (S * 2 * n <= nt && S < 16) S *= 2;
    HPT = (HP4 + S - 1) / S;          // hidden columns per phase-F thread
    HR = S * HPT;                     // rows of the W1 copy (zero past H)
    HS = (HR + 3) / 4 * 4;            // LDS row stride of A and delta1
    if (HS % 8 == 0) HS += 4;         // rows 4 floats apart modulo 8: no b128 bank aliasing
  }
  // float offsets of each LDS region (all multiples of 4)
  __host__ __device__ int xs() const { return 0; }               // X|1     [N][DP]
  __host__ __device__ int w1() const { return xs() + N * DP; }   // W1|b1   [HR][DP] master
  __host__ __device__ int c1() const { return w1() + HR * DP; }  // its Kahan terms [H][DP]
  __host__ __device__ int w2() const { return c1() + H * DP; }   // W2|b2   [4][HS] master
  __host__ __device__ int c2() const { return w2() + 4 * HS; }   // its Kahan terms [4][HS]
  __host__ __device__ int a() const { return c2() + 4 * HS; }    // A|1     [N][HS]
  __host__ __device__ int d1() const { return a() + N * HS; }    // delta1  [N][HS]
  __host__ __device__ int d2() const { return d1() + N * HS; }   // delta2  [N][4]
  __host__ __device__ int ts() const { return d2() + N * 4; }    // T       [N][4]
  __host__ __device__ int red() const { return ts() + N * 4; }   // per-wave loss partials
  __host__ __device__ int total() const { return red() + 16; }
};

template <int NT>
__global__ __launch_bounds__(NT) void k_small_train(
    const mlp_batch_item *__restrict__ items, mlp_batch_item one, int D, int K,
    const float *__restrict__ X, const float *__restrict__ T, float *__restrict__ theta,
    float *__restrict__ comp, int epochs, float *__restrict__ loss_hist) {
  constexpr int HPTM = (72 * 128 + NT - 1) / NT;  // max hidden columns per phase-F thread
  constexpr int DPM = 52;                          // max padded feature columns (D <= 48)
  constexpr int CM = 8;                            // max lanes sharing a phase-G tile
  const mlp_batch_item it = items ? items[blockIdx.x] : one;
  const int N = it.n_rows, H = it.n_hidden;
  const float lr = it.lr;
  const SmallLayout L(N, H, D, K, NT);
  const int DP = L.DP, HA = L.HA, HS = L.HS, S = L.S, HPT = L.HPT, HR = L.HR;
  const int tid = threadIdx.x;

  extern __shared__ float4 smem4[];
  float *sm = reinterpret_cast<float *>(smem4);
  float *Xs = sm + L.xs();
  float *W1s = sm + L.w1();
  float *C1s = sm + L.c1();
  float *W2s = sm + L.w2();
  float *C2s = sm + L.c2();
  float *As = sm + L.a();
  float *D1s = sm + L.d1();
  float *D2s = sm + L.d2();
  float *Ts = sm + L.ts();
  float *red = sm + L.red();

  const float *Xg = X + it.x_off * D;
  const float *Tg = T + it.x_off * K;
  float *P = theta + it.p_off;
  float *Cp = comp ? comp + it.p_off : nullptr;
  const bool compensated = Cp != nullptr;
  const int oB1 = H * D, oW2 = oB1 + H, oB2 = oW2 + K * H;

  // ---- stage rows, targets, parameters and compensation (coalesced);
  //      zero every padding entry that a later read may touch
  for (int i = tid; i < N * DP; i += NT) {
    int r = i / DP, c = i - r * DP;
    Xs[i] = c < D ? Xg[(int64_t)r * D + c] : (c == D ? 1.0f : 0.0f);
  }
  for (int i = tid; i < N * 4; i += NT) {
    int r = i >> 2, k = i & 3;
    Ts[i] = k < K ? Tg[(int64_t)r * K + k] : 0.0f;
  }
  for (int i = tid; i < HR * DP; i += NT) {
    int h = i / DP, c = i - h * DP;
    float v = 0.0f, cv = 0.0f;
    if (h < H && c <= D) {
      int o = c < D ? h * D + c : oB1 + h;
      v = P[o];
      cv = compensated ? Cp[o] : 0.0f;
    }
    W1s[i] = v;
    if (h < H) C1s[i] = cv;
  }
  for (int i = tid; i < 4 * HS; i += NT) {
    int k = i / HS, h = i - k * HS;
    float v = 0.0f, cv = 0.0f;
    if (k < K && h <= H) {
      int o = h < H ? oW2 + k * H + h : oB2 + k;
      v = P[o];
      cv = compensated ? Cp[o] : 0.0f;
    }
    W2s[i] = v;
    C2s[i] = cv;
  }
  for (int i = tid; i < 2 * N * HS; i += NT) As[i] = 0.0f;  // As and D1s are adjacent
  __syncthreads();

  // ---- phase-G tile ownership (fixed for the whole run)
  const int nTD = DP / 4;
  const int T1 = ((H + 3) / 4) * nTD;  // tiles of [W1 b1]: 4 hidden x 4 columns
  const int T2 = (HA + 3) / 4;         // tiles of [W2 b2]: 4 outputs x 4 hidden(+bias)
  int C = 1;
  while (C * 2 <= CM && (T1 + T2) * C * 2 <= NT && C * 2 <= N) C *= 2;
  const int tile = tid / C, chunk = tid - tile * C;
  const bool g1 = tile < T1, g2 = !g1 && tile < T1 + T2;
  const bool owner = chunk == 0 && (g1 || g2);
  int th = 0, td = 0, tj = 0;
  if (g1) { th = tile / nTD; td = tile - th * nTD; }
  if (g2) tj = tile - T1;

  // ---- phase-F row ownership
  const int r = tid / S, s = tid - r * S;
  const bool row_on = r < N;
  const int hbeg = s * HPT;
  float tr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) tr[k] = row_on ? Ts[r * 4 + k] : 0.0f;
  const float dscale = 2.0f / (float)(N * K);
  const float inv_nk = 1.0f / (float)(N * K);

  for (int e = 0; e < epochs; ++e) {
    // ============================ phase F
    float sq = 0.0f;
    if (row_on) {
      float a[HPTM];
#pragma unroll
      for (int j = 0; j < HPTM; ++j) a[j] = 0.0f;
      const float4 *xr = reinterpret_cast<const float4 *>(Xs + r * DP);
      const float4 *wr = reinterpret_cast<const float4 *>(W1s + hbeg * DP);
      const int dp4 = DP / 4;
#pragma unroll
      for (int c4 = 0; c4 < DPM / 4; ++c4) {
        if (c4 < dp4) {
          const float4 xv = xr[c4];
#pragma unroll
          for (int j = 0; j < HPTM; ++j) {
            if (j < HPT) {
              const float4 wv = wr[j * dp4 + c4];
              a[j] = fmaf(xv.x, wv.x, a[j]);
              a[j] = fmaf(xv.y, wv.y, a[j]);
              a[j] = fmaf(xv.z, wv.z, a[j]);
              a[j] = fmaf(xv.w, wv.w, a[j]);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < HPTM; ++j) {
        const int h = hbeg + j;
        a[j] = h < H ? sigmoid(a[j]) : (h == H ? 1.0f : 0.0f);  // column H: bias of layer 2
      }
      float z2[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float acc = 0.0f;
        if (k < K) {
          const float *w2r = W2s + k * HS + hbeg;
#pragma unroll
          for (int j = 0; j < HPTM; ++j)
            if (j < HPT) acc = fmaf(a[j], w2r[j], acc);
        }
        z2[k] = acc;
      }
      for (int off = 1; off < S; off <<= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) z2[k] += __shfl_xor(z2[k], off, kWave);
      float d2[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        d2[k] = 0.0f;
        if (k < K) {
          float y = sigmoid(z2[k]);
          float err = y - tr[k];
          sq = fmaf(err, err, sq);
          d2[k] = dscale * err * y * (1.0f - y);
        }
      }
      if (s) sq = 0.0f;  // each row's error is counted once
      float *arow = As + r * HS + hbeg;
      float *drow = D1s + r * HS + hbeg;
#pragma unroll
      for (int j = 0; j < HPTM; ++j) {
        const int h = hbeg + j;
        if (j < HPT) {
          float bp = 0.0f;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < K) bp = fmaf(d2[k], W2s[k * HS + h], bp);
          arow[j] = a[j];
          drow[j] = h < H ? bp * a[j] * (1.0f - a[j]) : 0.0f;
        }
      }
      if (!s) reinterpret_cast<float4 *>(D2s)[r] = make_float4(d2[0], d2[1], d2[2], d2[3]);
    }
    if (loss_hist) {
      sq = wave_sum(sq);
      if ((tid & (kWave - 1)) == 0) red[tid / kWave] = sq;
    }
    __syncthreads();

    // ============================ phase G
    if (loss_hist && tid == 0) {
      float tot = 0.0f;
      for (int q = 0; q < NT / kWave; ++q) tot += red[q];
      loss_hist[(int64_t)blockIdx.x * epochs + e] = tot * inv_nk;
    }
    float acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
    if (g1 || g2) {
      const float *pa = g1 ? D1s + 4 * th : D2s;         // left factor: delta1 cols or delta2
      const float *pb = g1 ? Xs + 4 * td : As + 4 * tj;  // right factor: x cols or a cols
      const int sa = g1 ? HS : 4, sb = g1 ? DP : HS;
      int n = chunk;
      for (; n + C < N; n += 2 * C) {
        const float4 u0 = *reinterpret_cast<const float4 *>(pa + n * sa);
        const float4 v0 = *reinterpret_cast<const float4 *>(pb + n * sb);
        const float4 u1 = *reinterpret_cast<const float4 *>(pa + (n + C) * sa);
        const float4 v1 = *reinterpret_cast<const float4 *>(pb + (n + C) * sb);
        const float uu0[4] = {u0.x, u0.y, u0.z, u0.w}, vv0[4] = {v0.x, v0.y, v0.z, v0.w};
        const float uu1[4] = {u1.x, u1.y, u1.z, u1.w}, vv1[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[i * 4 + j] = fmaf(uu0[i], vv0[j], acc[i * 4 + j]);
            acc[i * 4 + j] = fmaf(uu1[i], vv1[j], acc[i * 4 + j]);
          }
      }
      if (n < N) {
        const float4 u0 = *reinterpret_cast<const float4 *>(pa + n * sa);
        const float4 v0 = *reinterpret_cast<const float4 *>(pb + n * sb);
        const float uu0[4] = {u0.x, u0.y, u0.z, u0.w}, vv0[4] = {v0.x, v0.y, v0.z, v0.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i * 4 + j] = fmaf(uu0[i], vv0[j], acc[i * 4 + j]);
      }
    }
    for (int off = C / 2; off >= 1; off >>= 1)  // fixed butterfly over the tile's C lanes
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += __shfl_xor(acc[q], off, kWave);
    if (owner) {
      if (g1) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int h = 4 * th + i, d = 4 * td + j;
            if (h < H && d <= D) {
              float wv = W1s[h * DP + d], cv = C1s[h * DP + d];
              gd_update(wv, cv, lr, acc[i * 4 + j], compensated);
              W1s[h * DP + d] = wv;
              C1s[h * DP + d] = cv;
            }
          }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int k = i, h = 4 * tj + j;
            if (k < K && h <= H) {
              float wv = W2s[k * HS + h], cv = C2s[k * HS + h];
              gd_update(wv, cv, lr, acc[i * 4 + j], compensated);
              W2s[k * HS + h] = wv;
              C2s[k * HS + h] = cv;
            }
          }
      }
    }
    __syncthreads();
  }

  // ---- write the trained parameters (and compensation) back once
  for (int i = tid; i < H * DP; i += NT) {
    int h = i / DP, c = i - h * DP;
    if (c <= D) {
      int o = c < D ? h * D + c : oB1 + h;
      P[o] = W1s[i];
      if (compensated) Cp[o] = C1s[i];
    }
  }
  for (int i = tid; i < 4 * HS; i += NT) {
    int k = i / HS, h = i - k * HS;
    if (k < K && h <= H) {
      int o = h < H ? oW2 + k * H + h : oB2 + k;
      P[o] = W2s[i];
      if (compensated) Cp[o] = C2s[i];
    }
  }
}

template <int NT>
hipError_t launch_one(const mlp_batch_item *items, mlp_batch_item one, int n_nets, int n_in,
                      int n_out, size_t lds, const float *X, const float *T, float *theta,
                      float *comp, int epochs, float *loss_hist, hipStream_t s) {
  auto kern = k_small_train<NT>;
  hipError_t e = hipFuncSetAttribute((const void *)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n_nets), dim3(NT), lds, s, items, one, n_in, n_out, X, T, theta,
                     comp, epochs, loss_hist);
  return hipGetLastError();
}

}  // namespace mlpk

namespace mlph {

size_t small_lds_bytes(int n_rows, int n_hidden, int n_in, int threads) {
  mlpk::SmallLayout L(n_rows, n_hidden, n_in, 4, threads);
  return sizeof(float) * (size_t)L.total();
}

int small_threads(int n_nets, int hint) {
  if (hint == 256 || hint == 512 || hint == 1024) return hint;
  return n_nets <= 64 ? 1024 : 256;
}

size_t small_launch_lds_bytes(int max_rows, int max_hidden, int n_in, int threads) {
  // The layout grows with N and H but also depends on the phase-F split S,
  // which shrinks as N grows; bound it over every N up to max_rows.
  size_t lds = 0;
  for (int n = 1; n <= max_rows; ++n) lds = std::max(lds, small_lds_bytes(n, max_hidden, n_in, threads));
  return lds;
}

hipError_t launch_small_train(const mlp_batch_item *items, mlp_batch_item one, int n_nets,
                              int n_in, int n_out, int max_rows, int max_hidden, const float *X,
                              const float *T, float *theta, float *comp, int epochs,
                              float *loss_hist, int threads, hipStream_t s) {
  // One net (or a few) alone on the chip: 1024 threads shorten each epoch's
  // critical path.  Many nets: 256 threads per net, several nets per CU.
  const size_t lds = small_launch_lds_bytes(max_rows, max_hidden, n_in, threads);
  if (threads == 1024)
    return mlpk::launch_one<1024>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs,
                                  loss_hist, s);
  if (threads == 512)
    return mlpk::launch_one<512>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs,
                                 loss_hist, s);
  return mlpk::launch_one<256>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs,
                               loss_hist, s);
}

}  // namespace mlph
