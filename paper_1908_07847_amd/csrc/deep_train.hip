// Fused full-batch trainer for networks with several hidden layers: section
// 2.2's loop (feed forward layer by layer, the error, backpropagation from
// the top layer down, every layer's update) for L weight layers, the whole
// run in one launch of one workgroup with the rows, targets, activations,
// deltas and parameters resident in LDS.
//
// Per epoch, separated by workgroup barriers:
//   forward, one phase per layer: lane (row r, units o and o + half) forms
//     z = b_l[o] + sum_i A_l[r][i] W_l[o][i] and applies the hidden
//     activation (the sigmoid of Equation 1 or tanh) or, on the top layer,
//     the sigmoid; rows are the fast index across lanes, so the weight row
//     is a broadcast read and the activation rows (odd strides) hit
//     distinct banks;
//   error: the mean squared error's terms and the top delta
//     2 (y - t) / (n K) * y (1 - y), the loss summed wave by wave in a
//     fixed order;
//   backward, one phase per layer, top down: the gradient of W_l and b_l as
//     sums over rows split into RS fixed row segments (one partial per
//     segment, so several lanes share a long sum), and, below the top layer,
//     the delta of the layer below through the pre-update W_l times the
//     slope of its activation;
//   update: the RS partials of each parameter added in segment order, then
//   theta <- theta - lr g (Kahan-compensated when a compensation array is
//   given) for every layer at once.
// All sums run in fixed orders, so a run is bitwise repeatable.
#include <algorithm>

#include "deep.hpp"
#include "mlp_device.hpp"

namespace mlpk {

using mlph::DeepPlan;

// x / d and x mod d for 0 <= x < 2^20, 1 <= d, from the float reciprocal
// inv = 1/d: the estimate is within one of the quotient (relative error
// below 2^-22 on a quotient below 2^20) and one correction step makes it
// exact.  About eight VALU operations instead of an integer division.
__device__ __forceinline__ int div_small(int x, int d, float inv, int &rem) {
  int q = (int)((float)x * inv);
  int r = x - q * d;
  if (r < 0) {
    q -= 1;
    r += d;
  } else if (r >= d) {
    q += 1;
    r -= d;
  }
  rem = r;
  return q;
}

template <int ACT>
__global__ __launch_bounds__(mlph::kDeepThreads) void k_deep_train(
    DeepPlan p, const float *__restrict__ X, const float *__restrict__ T, float *__restrict__ theta,
    float *__restrict__ comp, float lr, int epochs, float *__restrict__ loss_hist) {
  constexpr int NT = mlph::kDeepThreads, NW = NT / kWave;
  extern __shared__ float4 smem4[];
  float *sm = reinterpret_cast<float *>(smem4);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = p.L, n = p.n, P = p.P, K = p.w[L], sK = p.sa[L], sd = p.sd;
  const bool compensated = comp != nullptr;

  // ---- stage rows, targets, parameters and compensation terms (coalesced)
  {
    const int d = p.w[0], s = p.sa[0];
    for (int i = tid; i < n * d; i += NT) {
      const int r = i / d, c = i - r * d;
      sm[p.aoff[0] + r * s + c] = X[i];
    }
  }
  for (int i = tid; i < n * K; i += NT) {
    const int r = i / K, k = i - r * K;
    sm[p.toff + r * sK + k] = T[i];
  }
  // a column of ones after every layer input's row: the bias is the last
  // column of the gradient's row sums
  for (int i = tid; i < n * L; i += NT) {
    const int l = i / n, r = i - l * n;
    sm[p.aoff[l] + r * p.sa[l] + p.w[l]] = 1.0f;
  }
  for (int q = tid; q < P; q += NT) {
    sm[p.th + q] = theta[q];
    sm[p.cp + q] = compensated ? comp[q] : 0.0f;
  }
  __syncthreads();

  const float dscale = 2.0f / ((float)n * (float)K);
  const float inv_nk = 1.0f / ((float)n * (float)K);
  float *Dtop = sm + ((L & 1) ? p.d1 : p.d0);

  for (int e = 0; e < epochs; ++e) {
    // ======================= feed forward
    for (int l = 0; l < L; ++l) {
      const int wi = p.w[l], wo = p.w[l + 1], si = p.sa[l], so = p.sa[l + 1];
      const float *A = sm + p.aoff[l];
      const float *W = sm + p.th + p.poff[l];
      const float *b = W + wo * wi;
      float *Y = sm + p.aoff[l + 1];
      const bool hidden = l < L - 1;
      // units in pairs (o0, o0 + hO) of one row: the row's inputs load once
      const int hO = (wo + 1) >> 1;
      const float inv_n = 1.0f / (float)n;
      for (int idx = tid; idx < n * hO; idx += NT) {
        int r;
        const int o0 = div_small(idx, n, inv_n, r);
        const int o1 = o0 + hO, o1r = min(o1, wo - 1);   // o1 = wo only when wo is odd: dropped
        const float *a = A + r * si, *w0 = W + o0 * wi, *w1 = W + o1r * wi;
        float z0 = b[o0], z1 = b[o1r];
#pragma unroll 8
        for (int i = 0; i < wi; ++i) {
          const float av = a[i];
          z0 = fmaf(av, w0[i], z0);
          z1 = fmaf(av, w1[i], z1);
        }
        Y[r * so + o0] = (hidden && ACT == 1) ? tanhf(z0) : sigmoid(z0);
        if (o1 < wo) Y[r * so + o1] = (hidden && ACT == 1) ? tanhf(z1) : sigmoid(z1);
      }
      __syncthreads();
    }

    // ======================= error and the top layer's delta
    {
      const float *Y = sm + p.aoff[L], *Ts = sm + p.toff;
      float part = 0.0f;
      const float inv_k = 1.0f / (float)K;
      for (int idx = tid; idx < n * K; idx += NT) {
        int k;
        const int r = div_small(idx, K, inv_k, k);
        const float y = Y[r * sK + k], d = y - Ts[r * sK + k];
        part = fmaf(d, d, part);
        Dtop[r * sd + k] = (dscale * d) * (y * (1.0f - y));
      }
      part = wave_sum(part);
      if (lane == 0) sm[p.red + wave] = part;
      __syncthreads();
      if (loss_hist && tid == 0) {
        float t = 0.0f;
        for (int w = 0; w < NW; ++w) t += sm[p.red + w];
        loss_hist[e] = t * inv_nk;
      }
    }

    // ======================= backpropagation, top layer first
    for (int l = L - 1; l >= 0; --l) {
      const int wi = p.w[l], wo = p.w[l + 1], si = p.sa[l];
      const float *A = sm + p.aoff[l];
      const float *W = sm + p.th + p.poff[l];
      const float *Dn = sm + (((l + 1) & 1) ? p.d1 : p.d0);
      float *Dl = sm + ((l & 1) ? p.d1 : p.d0);
      // the gradient's columns c = 0 .. wi (c = wi: the bias) in pairs (c, c + h)
      const int h = (wi + 2) >> 1, nW = wo * h, nG = p.RS * nW, nD = l > 0 ? n * wi : 0;
      float *G = sm + p.gr + p.poff[l];
      const float inv_nw = 1.0f / (float)nW, inv_h = 1.0f / (float)h, inv_wi = 1.0f / (float)wi;
      for (int idx = tid; idx < nG + nD; idx += NT) {
        if (idx < nG) {
          // segment sg of the row sums of parameters (o, c0) and (o, c1);
          // column wi is the bias (its input is the column of ones)
          int k, c0;
          const int sg = div_small(idx, nW, inv_nw, k);
          const int o = div_small(k, h, inv_h, c0);
          const int c1 = c0 + h, c1r = min(c1, wi);   // c1 = wi + 1 only when wi + 1 is odd: dropped
          const int r0 = sg * p.seg, r1 = min(n, r0 + p.seg);
          float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll 8
          for (int r = r0; r < r1; ++r) {
            const float d = Dn[r * sd + o];
            const float *ar = A + r * si;
            acc0 = fmaf(d, ar[c0], acc0);
            acc1 = fmaf(d, ar[c1r], acc1);
          }
          G[sg * P + (c0 < wi ? o * wi + c0 : wo * wi + o)] = acc0;
          if (c1 <= wi) G[sg * P + (c1 < wi ? o * wi + c1 : wo * wi + o)] = acc1;
        } else {
          // delta of layer l's input units (a hidden layer) at row r
          const int j = idx - nG;
          int i;
          const int r = div_small(j, wi, inv_wi, i);
          const float *dr = Dn + r * sd;
          float acc = 0.0f;
#pragma unroll 8
          for (int o = 0; o < wo; ++o) acc = fmaf(dr[o], W[o * wi + i], acc);
          const float a = A[r * si + i];
          Dl[r * sd + i] = acc * (ACT == 1 ? 1.0f - a * a : a * (1.0f - a));
        }
      }
      __syncthreads();
    }

    // ======================= update every layer at once
    for (int q = tid; q < P; q += NT) {
      float g = sm[p.gr + q];
      for (int sg = 1; sg < p.RS; ++sg) g += sm[p.gr + sg * P + q];
      float w = sm[p.th + q], c = sm[p.cp + q];
      gd_update(w, c, lr, g, compensated);
      sm[p.th + q] = w;
      sm[p.cp + q] = c;
    }
    __syncthreads();
  }

  // ---- write the trained parameters (and compensation) back once
  for (int q = tid; q < P; q += NT) {
    theta[q] = sm[p.th + q];
    if (compensated) comp[q] = sm[p.cp + q];
  }
}

}  // namespace mlpk

namespace mlph {

bool deep_plan(int L, const int32_t *widths, int64_t n, size_t lds_max, DeepPlan *p) {
  if (L < 1 || L > kDeepMaxLayers || n < 1 || n > (1 << 20)) return false;
  for (int l = 0; l <= L; ++l)
    if (widths[l] < 1 || widths[l] > kDeepMaxWidth) return false;
  DeepPlan q{};
  q.L = L;
  q.n = (int)n;
  int64_t P = 0;
  for (int l = 0; l <= L; ++l) {
    q.w[l] = widths[l];
    q.sa[l] = (widths[l] + 1) | 1;   // room for the column of ones
    q.poff[l] = (int)P;
    if (l < L) P += (int64_t)widths[l + 1] * widths[l] + widths[l + 1];
  }
  const int64_t cap = (int64_t)(lds_max / sizeof(float));
  if (P > cap) return false;
  q.P = (int)P;
  int64_t o = 0;
  for (int l = 0; l <= L; ++l) {
    q.aoff[l] = (int)std::min<int64_t>(o, cap);
    o += n * q.sa[l];
    if (o > cap) return false;
  }
  q.toff = (int)o;
  o += n * q.sa[L];
  int sd = 1;
  for (int l = 1; l <= L; ++l) sd = std::max(sd, q.sa[l]);
  q.sd = sd;
  q.d0 = (int)std::min<int64_t>(o, cap);
  o += n * sd;
  q.d1 = (int)std::min<int64_t>(o, cap);
  o += n * sd;
  q.th = (int)std::min<int64_t>(o, cap);
  o += P;
  q.cp = (int)std::min<int64_t>(o, cap);
  o += P;
  q.red = (int)std::min<int64_t>(o, cap);
  o += kDeepThreads / 64;   // one slot per wave
  if (o > cap) return false;
  q.gr = (int)o;
  // the most row segments (8, 4, 2 or 1, each of at least 8 rows) that fit;
  // a segment's length is a multiple of 8 rows (the unroll of its sums) and
  // the last one takes what is left
  for (int rs = 8; rs >= 1; rs >>= 1) {
    const int64_t seg = ((n + rs - 1) / rs + 7) / 8 * 8;
    if (rs > 1 && (n + rs - 1) / rs < 8) continue;
    if (o + rs * P <= cap) {
      q.RS = rs;
      q.seg = (int)seg;
      q.total = (int)(o + rs * P);
      *p = q;
      return true;
    }
  }
  return false;
}

hipError_t launch_deep_train(const DeepPlan &p, int act, const float *X, const float *T, float *theta,
                             float *comp, float lr, int epochs, float *loss_hist, hipStream_t s) {
  const size_t lds = (size_t)p.total * sizeof(float);
  const void *kern = act == 1 ? (const void *)mlpk::k_deep_train<1> : (const void *)mlpk::k_deep_train<0>;
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (act == 1)
    hipLaunchKernelGGL(mlpk::k_deep_train<1>, dim3(1), dim3(kDeepThreads), lds, s, p, X, T, theta, comp, lr,
                       epochs, loss_hist);
  else
    hipLaunchKernelGGL(mlpk::k_deep_train<0>, dim3(1), dim3(kDeepThreads), lds, s, p, X, T, theta, comp, lr,
                       epochs, loss_hist);
  return hipGetLastError();
}

}  // namespace mlph
