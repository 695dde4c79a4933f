// Small-network trainer: one workgroup trains one network, full batch, for
// all epochs in a single launch (arxiv 1908.07847, section 2.2: feed
// forward, error, backpropagation, gradient-descent update, repeated for a
// number of epochs).
//
// The net lives in LDS for the whole run: its rows X with a constant-1
// column (so b1 is the last column of W1), the targets, W1|b1, W2 and b2.
// HBM is read once at the start and written once at the end.  Each of the
// NW waves owns every NW-th 16-row tile of the batch and, per epoch:
//
//   z1^T = [W1 b1] [X 1]^T     v_mfma_f32_16x16x4_f32, M = hidden, N = rows
//   a = sigma(z1), slope = a (1 - a) (as e^-z a^2), kept in registers in the
//       MFMA accumulator layout (lane: 1 row x 4 hidden units per 16x16 tile)
//   z2 = a W2^T + b2           per lane over its hidden units, then a
//                              reduce-scatter over the lanes of the row, so
//                              that lane (row n, group g) holds output g of
//                              row n and every lane evaluates one sigmoid
//   y = sigma(z2), delta2 = 2 (y - t) / (N K) . y (1 - y)
//   delta1^T = W2^T delta2^T   v_mfma_f32_16x16x4_f32 (the pre-update W2;
//                              the contraction over the <= 4 outputs is one
//                              instruction), times the slope
//   gW2^T += a^T delta2        v_mfma_f32_16x16x4_f32, K = the tile's rows
//   gW1 += delta1^T [X 1]      v_mfma_f32_16x16x4_f32, M = hidden, N = features,
//                              K = the tile's rows
//   gb2 += sum delta2          lane partials
//
// a, delta1 and delta2 pass through wave-private LDS tiles where a
// contraction needs them transposed.
//
// After a barrier the NW wave partials of every parameter are summed in wave
// order (bitwise repeatable) and the owner thread applies the update to the
// master copy in LDS, with its Kahan compensation term kept in registers;
// a second barrier publishes the new weights.  Padded rows carry zero X (so
// zero delta) and padded hidden units zero W2 (so zero delta1).
//
// Limits: N <= 128 rows, H <= 64, D <= 48, K <= 4.
#include <algorithm>
#include <type_traits>

#include "mlp_device.hpp"

namespace mlpk {

typedef float f32x4_s __attribute__((ext_vector_type(4)));

// The value of v in lane l of the wave (uniform result).
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// LDS plan (floats).
struct SmallLayout {
  int N, H, D, K, NW, NP, NPT, DA, DK, DN, XS, HP, HT, FT, PW;
  __host__ __device__ SmallLayout(int n, int h, int d, int k, int nw)
      : N(n), H(h), D(d), K(k), NW(nw) {
    NP = (n + 15) / 16 * 16;  // rows padded to 16-row tiles
    NPT = NP / 16;
    DA = d + 1;               // features + the constant-1 column
    DK = (DA + 3) / 4 * 4;    // contraction length of z1 (steps of 4)
    DN = (DA + 15) / 16 * 16; // feature tiles of gW1
    FT = DN / 16;
    XS = DN + 2;              // row stride of X and W1: 16 rows of a tile hit distinct banks
    HP = (h + 15) / 16 * 16;  // hidden units padded to 16-unit tiles
    HT = HP / 16;
    PW = HP * DN + 4 * HP + 4 + 4;  // one wave's partials: gW1 | gW2 | gb2 | loss
  }
  __host__ __device__ int xs() const { return 0; }                  // [NP][XS]
  __host__ __device__ int w1() const { return xs() + NP * XS; }     // [HP][XS] master W1|b1
  __host__ __device__ int w2() const { return w1() + HP * XS; }     // [4][HP]  master W2
  __host__ __device__ int b2() const { return w2() + 4 * HP; }      // [4]      master b2
  __host__ __device__ int ts() const { return b2() + 4; }           // [NP][4]  targets
  __host__ __device__ int dst() const { return ts() + NP * 4; }     // [NW][16][16] a / delta1 staging
  __host__ __device__ int dd() const { return dst() + NW * 256; }   // [NW][16][4] delta2 staging
  __host__ __device__ int part() const { return dd() + NW * 64; }   // [NW][PW] partials
  __host__ __device__ int vs() const { return part() + NW * PW; }   // [P] velocity (momentum only)
  __host__ __device__ int total(bool mom = false) const {
    return vs() + (mom ? (H * (D + 1) + K * H + K + 3) / 4 * 4 : 0);
  }
};

// Training variants (the paper's method is act 0 without momentum):
// hidden activation act (0 sigma, 1 tanh); heavy-ball momentum with rate mu
// when vel (the velocity [P], packed order, of a single net) is not null.
struct SmallVariant {
  int act;
  float mu;
  float *vel;
};

// KO: outputs the output-layer code runs over (K <= KO; 3 covers K <= 3).
// ACT: the hidden activation (0 sigma, 1 tanh), fixed per instance so the
// paper's sigmoid network carries no branch for the variant.
template <int NW, int HTM, int KO, int ACT>
__global__ __launch_bounds__(NW * 64) void k_small_train(
    const mlp_batch_item *__restrict__ items, mlp_batch_item one, int D, int K,
    const float *__restrict__ X, const float *__restrict__ T, float *__restrict__ theta,
    float *__restrict__ comp, int epochs, float *__restrict__ loss_hist, SmallVariant var) {
  constexpr int NT = NW * 64;
  constexpr int PMAX = 48 * 64 + 64 + 64 * 4 + 4;   // largest parameter count
  constexpr int JM = (PMAX + NT - 1) / NT;          // parameters per thread
  const mlp_batch_item it = items ? items[blockIdx.x] : one;
  const int N = it.n_rows, H = it.n_hidden;
  const float lr = it.lr;
  const SmallLayout L(N, H, D, K, NW);
  const int XS = L.XS, HP = L.HP, HT = L.HT, FT = L.FT, DN = L.DN, DK = L.DK, PW = L.PW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;

  extern __shared__ float4 smem4[];
  float *sm = reinterpret_cast<float *>(smem4);
  float *Xs = sm + L.xs();
  float *W1s = sm + L.w1();
  float *W2s = sm + L.w2();
  float *b2s = sm + L.b2();
  float *Ts = sm + L.ts();
  float *Dst = sm + L.dst() + wave * 256;
  float *Dd = sm + L.dd() + wave * 64;
  float *Part = sm + L.part();

  const float *Xg = X + it.x_off * D;
  const float *Tg = T + it.x_off * K;
  float *P = theta + it.p_off;
  float *Cp = comp ? comp + it.p_off : nullptr;
  const bool compensated = Cp != nullptr;
  const int D1 = D + 1;
  const int oB1 = H * D, oW2 = oB1 + H, oB2 = oW2 + K * H;
  const int nP = H * D1 + K * H + K;   // parameters, in update order: [W1 b1] rows, W2, b2

  // ---- stage rows, targets, parameters (coalesced); zero every padding entry
  for (int i = tid; i < L.NP * XS; i += NT) {
    const int r = i / XS, c = i - r * XS;
    Xs[i] = (r < N && c < D) ? Xg[(int64_t)r * D + c] : ((r < N && c == D) ? 1.0f : 0.0f);
  }
  for (int i = tid; i < L.NP * 4; i += NT) {
    const int r = i >> 2, k = i & 3;
    Ts[i] = (r < N && k < K) ? Tg[(int64_t)r * K + k] : 0.0f;
  }
  for (int i = tid; i < HP * XS; i += NT) {
    const int h = i / XS, c = i - h * XS;
    W1s[i] = (h < H && c < D) ? P[h * D + c] : ((h < H && c == D) ? P[oB1 + h] : 0.0f);
  }
  for (int i = tid; i < 4 * HP; i += NT) {
    const int k = i / HP, h = i - k * HP;
    W2s[i] = (k < K && h < H) ? P[oW2 + k * H + h] : 0.0f;
  }
  if (tid < 4) b2s[tid] = tid < K ? P[oB2 + tid] : 0.0f;
  // Kahan terms of the parameters this thread updates (q = tid + j*NT)
  // packed offset of parameter q (update order)
  auto packed = [&](int q) {
    if (q < H * D1) {
      const int h = q / D1, d = q - h * D1;
      return d < D ? h * D + d : oB1 + h;
    }
    if (q < H * D1 + K * H) return oW2 + (q - H * D1);
    return oB2 + (q - H * D1 - K * H);
  };
  float ccomp[JM];
#pragma unroll
  for (int j = 0; j < JM; ++j) {
    const int q = tid + j * NT;
    ccomp[j] = (compensated && q < nP) ? Cp[packed(q)] : 0.0f;
  }
  // momentum: the velocity lives in LDS in update order for the whole run
  float *Vs = sm + L.vs();
  if (var.vel)
    for (int q = tid; q < nP; q += NT) Vs[q] = var.vel[packed(q)];
  // LDS offsets of parameter q (update order): its partial within a wave's
  // block and its master copy.  Kept packed in registers across epochs when
  // a thread owns few parameters.
  auto offsets = [&](int q, int &po, int &mo) {
    if (q < H * D1) {
      const int h = q / D1, d = q - h * D1;
      po = h * DN + d;
      mo = L.w1() + h * XS + d;
    } else if (q < H * D1 + K * H) {
      const int o = q - H * D1, k = o / H, h = o - k * H;
      po = HP * DN + k * HP + h;
      mo = L.w2() + k * HP + h;
    } else {
      const int k = q - H * D1 - K * H;
      po = HP * DN + 4 * HP + k;
      mo = L.b2() + k;
    }
  };
  constexpr bool kKeepOfs = JM <= 8;
  int uofs[kKeepOfs ? JM : 1];
  if constexpr (kKeepOfs) {
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      const int q = tid + j * NT;
      int po = 0, mo = 0;
      if (q < nP) offsets(q, po, mo);
      uofs[j] = (po << 16) | mo;   // both below 2^16
    }
  }
  __syncthreads();

  const float dscale = 2.0f / (float)(N * K);
  const float inv_nk = 1.0f / (float)(N * K);

  for (int e = 0; e < epochs; ++e) {
    // ======================= rows of this wave: forward, deltas, partial gradients
    f32x4_s gacc[HTM][4];   // gW1 tiles [hidden][feature]
    f32x4_s g2acc[HTM];     // gW2^T tiles [hidden][output]
#pragma unroll
    for (int ht = 0; ht < HTM; ++ht) {
      g2acc[ht] = f32x4_s{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ft = 0; ft < 4; ++ft) gacc[ht][ft] = f32x4_s{0.f, 0.f, 0.f, 0.f};
    }
    float gb2 = 0.0f;   // output lg of this lane's rows
    float sq = 0.0f;

    for (int rt = wave; rt < L.NPT; rt += NW) {
      const int r0 = rt * 16;
      const int n = r0 + l16;   // this lane's row
      // z1^T tiles (M = hidden, N = rows): lane (row l16, group lg) holds
      // hidden units 4 lg .. 4 lg + 3 of each tile; a and its slope stay in
      // registers
      float av[HTM][4], sl[HTM][4];
#pragma unroll
      for (int ht = 0; ht < HTM; ++ht) {
#pragma unroll
        for (int i = 0; i < 4; ++i) { av[ht][i] = 0.0f; sl[ht][i] = 0.0f; }
        if (ht < HT) {
          f32x4_s z = {0.f, 0.f, 0.f, 0.f};
          const float *xa = Xs + (r0 + l16) * XS + lg;
          const float *wb = W1s + (ht * 16 + l16) * XS + lg;
          for (int k0 = 0; k0 < DK; k0 += 4)
            z = __builtin_amdgcn_mfma_f32_16x16x4f32(wb[k0], xa[k0], z, 0, 0, 0);
#pragma unroll
          for (int i = 0; i < 4; ++i) av[ht][i] = hidden_act(ACT, z[i], sl[ht][i]);
        }
      }
      // output layer: each lane's share of z2 (its 4 hidden units per tile)
      // for every output, then a reduce-scatter over the four row groups
      // (lanes n, n+16, n+32, n+48) leaves z2[n][lg] in lane (n, lg): every
      // lane evaluates one output of one row.  Padding hidden tiles read
      // tile 0's weights and multiply them by a zero activation.
      float zp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ht = 0; ht < HTM; ++ht) {
        const int hs = (ht < HT ? ht : 0) * 16 + 4 * lg;
#pragma unroll
        for (int k = 0; k < KO; ++k) {
          const f32x4_s w = *reinterpret_cast<const f32x4_s *>(W2s + k * HP + hs);
#pragma unroll
          for (int i = 0; i < 4; ++i) zp[k] = fmaf(av[ht][i], w[i], zp[k]);
        }
      }
      const bool hi2 = (lg & 2) != 0, hi1 = (lg & 1) != 0;
      float ka = hi2 ? zp[2] : zp[0], kb = hi2 ? zp[3] : zp[1];   // outputs kept
      const float sa = hi2 ? zp[0] : zp[2], sb = hi2 ? zp[1] : zp[3];
      ka += __shfl_xor(sa, 32, kWave);
      kb += __shfl_xor(sb, 32, kWave);
      const float z2 = (hi1 ? kb : ka) + __shfl_xor(hi1 ? ka : kb, 16, kWave);
      const int k = lg;
      const float y = sigmoid(z2 + b2s[k]);
      const bool on = k < K && n < N;
      const float err = on ? y - Ts[n * 4 + k] : 0.0f;
      sq = fmaf(err, err, sq);
      const float d2 = dscale * err * y * (1.0f - y);
      gb2 += d2;
      Dd[l16 * 4 + k] = d2;   // row-major [row][output] for the gW2 contraction
#pragma unroll
      for (int ht = 0; ht < HTM; ++ht) {
        if (ht < HT) {
          // gW2^T += a^T delta2 (M = hidden, N = outputs, K = the tile's
          // rows), a staged row-major through the wave's LDS tile
          *reinterpret_cast<f32x4_s *>(Dst + l16 * 16 + 4 * lg) =
              f32x4_s{av[ht][0], av[ht][1], av[ht][2], av[ht][3]};
          f32x4_s g2 = g2acc[ht];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const float dv = Dd[(4 * s + lg) * 4 + (l16 & 3)];
            g2 = __builtin_amdgcn_mfma_f32_16x16x4f32(Dst[(4 * s + lg) * 16 + l16], l16 < 4 ? dv : 0.0f,
                                                     g2, 0, 0, 0);
          }
          g2acc[ht] = g2;
          // delta1^T = W2^T delta2^T (the pre-update W2), times the slope
          const f32x4_s bp = __builtin_amdgcn_mfma_f32_16x16x4f32(
              W2s[lg * HP + ht * 16 + l16], d2, f32x4_s{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
          *reinterpret_cast<f32x4_s *>(Dst + l16 * 16 + 4 * lg) =
              f32x4_s{bp[0] * sl[ht][0], bp[1] * sl[ht][1], bp[2] * sl[ht][2], bp[3] * sl[ht][3]};
          // gW1 += delta1^T [X 1] on MFMA
          const float *da = Dst + lg * 16 + l16;
#pragma unroll
          for (int ft = 0; ft < 4; ++ft) {
            if (ft < FT) {
              const float *xb = Xs + (r0 + lg) * XS + ft * 16 + l16;
              f32x4_s g = gacc[ht][ft];
#pragma unroll
              for (int s = 0; s < 4; ++s)
                g = __builtin_amdgcn_mfma_f32_16x16x4f32(da[s * 64], xb[s * 4 * XS], g, 0, 0, 0);
              gacc[ht][ft] = g;
            }
          }
        }
      }
    }

    // ======================= wave partials to LDS
    float *pw = Part + wave * PW;
    // this lane's base in the block, opaque to the compiler each epoch: the
    // per-lane addresses below are then formed here (base + a wave-uniform
    // offset) instead of being kept live across the epoch loop, where the
    // wide instances would spill them
    int lbase = 4 * lg * DN + l16;
    asm volatile("" : "+v"(lbase));
#pragma unroll
    for (int ht = 0; ht < HTM; ++ht) {
      if (ht < HT) {
#pragma unroll
        for (int ft = 0; ft < 4; ++ft) {
          if (ft < FT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) pw[lbase + (ht * 16 + i) * DN + ft * 16] = gacc[ht][ft][i];
          }
        }
        // lane (output l16, group lg): hidden units 4 lg .. 4 lg + 3
        if (l16 < 4) *reinterpret_cast<f32x4_s *>(pw + HP * DN + l16 * HP + ht * 16 + 4 * lg) = g2acc[ht];
      }
    }
    gb2 = sum16(gb2);
    if (l16 == 0) pw[HP * DN + 4 * HP + lg] = gb2;
    // (the lane reads stay outside the branch: the row sums must be complete
    // in all four rows, not only in the lane that stores)
    sq = sum16(sq);
    const float sqw = (lane_value(sq, 0) + lane_value(sq, 16)) + (lane_value(sq, 32) + lane_value(sq, 48));
    if (lane == 0) pw[HP * DN + 4 * HP + 4] = sqw;
    __syncthreads();

    // ======================= sum the wave partials in order; update
    if (loss_hist && tid == 0) {
      float s = 0.0f;
      for (int w = 0; w < NW; ++w) s += Part[w * PW + HP * DN + 4 * HP + 4];
      loss_hist[(int64_t)blockIdx.x * epochs + e] = s * inv_nk;
    }
    if constexpr (kKeepOfs) {
      // the partial sums of a thread's first two parameters load
      // unconditionally (an unused slot reads offset 0), so both batches of
      // loads are in flight together
      float gs[JM];
#pragma unroll
      for (int j = 0; j < JM; ++j) {
        gs[j] = 0.0f;
        if (j < 2 || tid + j * NT < nP) {
          const int po = uofs[j] >> 16;
#pragma unroll
          for (int w = 0; w < NW; ++w) gs[j] += Part[w * PW + po];
        }
      }
#pragma unroll
      for (int j = 0; j < JM; ++j) {
        if (tid + j * NT < nP) {
          const int mo = uofs[j] & 0xffff;
          float wv = sm[mo], g = gs[j];
          if (var.vel) {   // heavy-ball momentum: v <- mu v + g, step along v
            g = fmaf(var.mu, Vs[tid + j * NT], g);
            Vs[tid + j * NT] = g;
          }
          gd_update(wv, ccomp[j], lr, g, compensated);
          sm[mo] = wv;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < JM; ++j) {
        const int q = tid + j * NT;
        if (q < nP) {
          int po, mo;
          offsets(q, po, mo);
          float g = 0.0f;
          for (int w = 0; w < NW; ++w) g += Part[w * PW + po];
          if (var.vel) {
            g = fmaf(var.mu, Vs[q], g);
            Vs[q] = g;
          }
          float wv = sm[mo];
          gd_update(wv, ccomp[j], lr, g, compensated);
          sm[mo] = wv;
        }
      }
    }
    __syncthreads();
  }

  // ---- write the trained parameters (and compensation) back once
#pragma unroll
  for (int j = 0; j < JM; ++j) {
    const int q = tid + j * NT;
    if (q < nP) {
      int o;
      float wv;
      if (q < H * D1) {
        const int h = q / D1, d = q - h * D1;
        o = d < D ? h * D + d : oB1 + h;
        wv = W1s[h * XS + d];
      } else if (q < H * D1 + K * H) {
        const int oo = q - H * D1, k = oo / H, h = oo - k * H;
        o = oW2 + oo;
        wv = W2s[k * HP + h];
      } else {
        const int k = q - H * D1 - K * H;
        o = oB2 + k;
        wv = b2s[k];
      }
      P[o] = wv;
      if (compensated) Cp[o] = ccomp[j];
    }
  }
  if (var.vel)
    for (int q = tid; q < nP; q += NT) var.vel[packed(q)] = Vs[q];
}

template <int NW, int HTM, int KO, int ACT>
hipError_t launch_one(const mlp_batch_item *items, mlp_batch_item one, int n_nets, int n_in,
                      int n_out, size_t lds, const float *X, const float *T, float *theta,
                      float *comp, int epochs, float *loss_hist, SmallVariant var, hipStream_t s) {
  auto kern = k_small_train<NW, HTM, KO, ACT>;
  hipError_t e = hipFuncSetAttribute((const void *)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n_nets), dim3(NW * 64), lds, s, items, one, n_in, n_out, X, T,
                     theta, comp, epochs, loss_hist, var);
  return hipGetLastError();
}

template <int NW, int ACT>
hipError_t launch_nw(int max_hidden, const mlp_batch_item *items, mlp_batch_item one, int n_nets,
                     int n_in, int n_out, size_t lds, const float *X, const float *T,
                     float *theta, float *comp, int epochs, float *loss_hist, SmallVariant var,
                     hipStream_t s) {
  // registers are sized for the widest hidden layer of the launch
  const int ht = (max_hidden + 15) / 16;
  if (n_out <= 3) {
    if (ht <= 1)
      return launch_one<NW, 1, 3, ACT>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, var, s);
    if (ht <= 2)
      return launch_one<NW, 2, 3, ACT>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, var, s);
    return launch_one<NW, 4, 3, ACT>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, var, s);
  }
  if (ht <= 1)
    return launch_one<NW, 1, 4, ACT>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, var, s);
  if (ht <= 2)
    return launch_one<NW, 2, 4, ACT>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, var, s);
  return launch_one<NW, 4, 4, ACT>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, var, s);
}


// ---------------------------------------------------------------------------
// Hidden-split form of the same trainer (the paper's sigmoid network, plain
// or compensated update): the NW waves of a workgroup split the hidden layer
// instead of the rows.  Wave w owns hidden tile w (units 16 w .. 16 w + 15)
// for every row of the net; waves past the net's last tile only pass the
// barriers.  Per epoch:
//   phase A (every 16-row tile): z1^T of the wave's tile on MFMA, kept in
//     registers for the epoch, and the tile's share of z2 (its
//     16 hidden units, reduce-scattered over the lanes of a row) to LDS;
//   one barrier;
//   phase B (every row tile): z2 = the tiles' shares summed in tile order
//     plus b2, y and delta2 (each wave forms them itself, so every wave holds
//     the same values), then for the wave's own units a and the slope again
//     from z1 (two sigmoids per element cost less than holding both),
//     gW2 += a^T delta2,
//     delta1 = (W2^T delta2) . slope with the pre-update W2, and
//     gW1 += delta1^T [X 1], all on MFMA and accumulated in registers;
//   the update: each wave applies its own W1 rows and W2 columns from the
//     registers that hold their gradients, the Kahan terms living in the same
//     lanes; b2 is kept and updated in registers by every wave alike (the
//     same delta2 sums), wave 0 writing it back at the end.
// A wave reads only its own W1 rows and W2 columns, the shares of consecutive
// epochs alternate between two buffers, and b2 is private to each wave, so
// one barrier per epoch suffices and no per-wave partial gradients exist:
// LDS holds X, the parameters and the shares only (the targets of a lane's
// rows stay in its registers for the run).  The row stride of X and W1 is
// DK + 2, the z1 contraction's length: the gW1 operand of the feature block
// past DK reads into the next row, which only feeds gradients of padding
// features that are never applied; so three 120-row, 64-unit nets share a CU.
// Limits: N <= 128 rows, H <= 16 NW <= 64, D <= 48, K <= KO <= 4.
struct HSplitLayout {
  int N, H, D, NW, KO, NP, NPT, DA, DK, DN, FT, XS, HP;
  __host__ __device__ HSplitLayout(int n, int h, int d, int nw, int ko)
      : N(n), H(h), D(d), NW(nw), KO(ko) {
    NP = (n + 15) / 16 * 16;
    NPT = NP / 16;
    DA = d + 1;
    DK = (DA + 3) / 4 * 4;
    DN = (DA + 15) / 16 * 16;
    FT = DN / 16;
    XS = DK + 2;
    HP = (h + 15) / 16 * 16;
  }
  __host__ __device__ int xs() const { return 0; }                 // [NP][XS] rows, ones column
  __host__ __device__ int w1() const { return xs() + NP * XS; }    // [HP][XS] W1 | b1
  __host__ __device__ int w2() const { return w1() + HP * XS; }    // [4][HP]
  __host__ __device__ int zs() const { return w2() + 4 * HP; }     // [2][NW][NP][KO] z2 shares
  __host__ __device__ int dst() const { return zs() + 2 * NW * NP * KO; }   // [NW][2][16][16] staging
  __host__ __device__ int dd() const { return dst() + NW * 512; }  // [NW][2][16][4] delta2 staging
  __host__ __device__ int total() const { return dd() + NW * 128 + 64; }   // + the over-read of the last X row
};

// At most 168 registers per lane (three waves per SIMD): three of the
// largest nets (52 KB of LDS each) share a CU.
template <int NW, int KO>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(3))) void k_small_hsplit(
    const mlp_batch_item *__restrict__ items, mlp_batch_item one, int D, int K,
    const float *__restrict__ X, const float *__restrict__ T, float *__restrict__ theta,
    float *__restrict__ comp, int epochs, float *__restrict__ loss_hist) {
  constexpr int NT = NW * 64;
  const mlp_batch_item it = items ? items[blockIdx.x] : one;
  const int N = it.n_rows, H = it.n_hidden;
  const float lr = it.lr;
  const HSplitLayout L(N, H, D, NW, KO);
  const int XS = L.XS, HP = L.HP, FT = L.FT, DK = L.DK, NP = L.NP, NPT = L.NPT;
  const int HTn = HP / 16;   // hidden tiles of this net
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16_0 = lane & 15, lg_0 = lane >> 4;
  int l16 = l16_0, lg = lg_0;

  extern __shared__ float4 smem4[];
  float *sm = reinterpret_cast<float *>(smem4);
  float *Xs = sm + L.xs();
  float *W1s = sm + L.w1();
  float *W2s = sm + L.w2();
  float *Zs = sm + L.zs();
  float *Dst = sm + L.dst() + wave * 512;   // two buffers: a pair of row tiles
  float *Dd = sm + L.dd() + wave * 128;

  const float *Xg = X + it.x_off * D;
  const float *Tg = T + it.x_off * K;
  float *P = theta + it.p_off;
  float *Cp = comp ? comp + it.p_off : nullptr;
  const bool compensated = Cp != nullptr;
  const int D1 = D + 1;
  const int oB1 = H * D, oW2 = oB1 + H, oB2 = oW2 + K * H;

  // ---- stage rows (with the ones column), targets, W1 | b1, W2; zero padding
  for (int i = tid; i < NP * XS; i += NT) {
    const int r = i / XS, c = i - r * XS;
    Xs[i] = (r < N && c < D) ? Xg[(int64_t)r * D + c] : ((r < N && c == D) ? 1.0f : 0.0f);
  }
  for (int i = tid; i < HP * XS; i += NT) {
    const int h = i / XS, c = i - h * XS;
    W1s[i] = (h < H && c < D) ? P[h * D + c] : ((h < H && c == D) ? P[oB1 + h] : 0.0f);
  }
  // the target of lane (row l16, output lg) of every row tile
  float tv[8];
#pragma unroll
  for (int rt = 0; rt < 8; ++rt) {
    const int n = rt * 16 + l16;
    tv[rt] = (n < N && lg < K) ? Tg[(int64_t)n * K + lg] : 0.0f;
  }
  for (int i = tid; i < 4 * HP; i += NT) {
    const int k = i / HP, h = i - k * HP;
    W2s[i] = (k < K && h < H) ? P[oW2 + k * H + h] : 0.0f;
  }
  // this wave's tile and the parameters its lanes update: W1[h0 + 4 lg + i]
  // [16 ft + l16] (b1 is column D), W2[l16][h0 + 4 lg + i] for l16 < K, and
  // b2[lg] (every wave's own copy)
  const bool own = wave < HTn;
  const int h0 = wave * 16;
  float c1[4][4], c2[4];
#pragma unroll
  for (int ft = 0; ft < 4; ++ft)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = h0 + 4 * lg + i, d = 16 * ft + l16;
      c1[ft][i] = (compensated && own && h < H && d < D1) ? Cp[d < D ? h * D + d : oB1 + h] : 0.0f;
    }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int h = h0 + 4 * lg + i;
    c2[i] = (compensated && own && l16 < K && h < H) ? Cp[oW2 + l16 * H + h] : 0.0f;
  }
  float b2v = lg < K ? P[oB2 + lg] : 0.0f;
  float cb = (compensated && lg < K) ? Cp[oB2 + lg] : 0.0f;
  __syncthreads();

  const float dscale = 2.0f / (float)(N * K);
  const float inv_nk = 1.0f / (float)(N * K);

  for (int e = 0; e < epochs; ++e) {
    float *zs = Zs + (e & 1) * (NW * NP * KO);
    // the lane coordinates, opaque to the compiler each epoch: the per-lane
    // LDS addresses are formed here instead of being hoisted out of the
    // epoch loop and held (or spilled) for the whole run
    int l16 = l16_0, lg = lg_0;
    asm volatile("" : "+v"(l16), "+v"(lg));
    float zz[8][4];   // z1 of this wave's units, every row tile (a and the slope are re-formed from it)
    // ======================= phase A: a of this wave's tile, its share of z2
    // Row tiles go in pairs whose two z1 chains share the W1 operand and
    // interleave on the matrix cores (a lone last tile runs its own chain).
    if (own) {
      const float *wb = W1s + (h0 + l16) * XS + lg;
      auto finish = [&](auto rt_c, const f32x4_s &z) {
        constexpr int rt = decltype(rt_c)::value;
        float a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          zz[rt][i] = z[i];
          a[i] = sigmoid(z[i]);
        }
        float zp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < KO; ++k) {
          const f32x4_s w = *reinterpret_cast<const f32x4_s *>(W2s + k * HP + h0 + 4 * lg);
#pragma unroll
          for (int i = 0; i < 4; ++i) zp[k] = fmaf(a[i], w[i], zp[k]);
        }
        // reduce-scatter over the row's four lane groups: lane (row, lg)
        // ends with output lg of the row
        const bool hi2 = (lg & 2) != 0, hi1 = (lg & 1) != 0;
        float ka = hi2 ? zp[2] : zp[0], kb = hi2 ? zp[3] : zp[1];
        const float sa = hi2 ? zp[0] : zp[2], sb = hi2 ? zp[1] : zp[3];
        ka += __shfl_xor(sa, 32, kWave);
        kb += __shfl_xor(sb, 32, kWave);
        const float share = (hi1 ? kb : ka) + __shfl_xor(hi1 ? ka : kb, 16, kWave);
        if (lg < KO) zs[(wave * NP + rt * 16 + l16) * KO + lg] = share;
      };
      auto pair = [&](auto r0_c) {
        constexpr int r0 = decltype(r0_c)::value;
        const float *xa = Xs + (r0 * 16 + l16) * XS + lg;
        if (r0 + 1 < NPT) {
          const float *xb = xa + 16 * XS;
          f32x4_s za = {0.f, 0.f, 0.f, 0.f}, zb = {0.f, 0.f, 0.f, 0.f};
          for (int k0 = 0; k0 < DK; k0 += 4) {
            const float w = wb[k0];
            za = __builtin_amdgcn_mfma_f32_16x16x4f32(w, xa[k0], za, 0, 0, 0);
            zb = __builtin_amdgcn_mfma_f32_16x16x4f32(w, xb[k0], zb, 0, 0, 0);
          }
          finish(std::integral_constant<int, r0>{}, za);
          finish(std::integral_constant<int, r0 + 1>{}, zb);
        } else if (r0 < NPT) {
          f32x4_s za = {0.f, 0.f, 0.f, 0.f};
          for (int k0 = 0; k0 < DK; k0 += 4) za = __builtin_amdgcn_mfma_f32_16x16x4f32(wb[k0], xa[k0], za, 0, 0, 0);
          finish(std::integral_constant<int, r0>{}, za);
        }
      };
      pair(std::integral_constant<int, 0>{});
      pair(std::integral_constant<int, 2>{});
      pair(std::integral_constant<int, 4>{});
      pair(std::integral_constant<int, 6>{});
    }
    __syncthreads();
    if (!own) continue;
    // ======================= phase B: delta2, then this tile's gradients
    // Row tiles again go in pairs (two staging buffers), every product in
    // the order a tile-by-tile loop would issue it, so a pair gives the same
    // bits as its two tiles one after the other.
    f32x4_s gacc[4], g2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) gacc[ft] = f32x4_s{0.f, 0.f, 0.f, 0.f};
    float gb2 = 0.0f, sq = 0.0f;
    // delta2 of row tile rt in lane (row l16, output lg)
    auto delta2 = [&](auto rt_c) {
      constexpr int rt = decltype(rt_c)::value;
      const int n = rt * 16 + l16, k = lg;
      float z2 = 0.0f;
      if (k < KO)
        for (int w = 0; w < HTn; ++w) z2 += zs[(w * NP + n) * KO + k];
      const float y = sigmoid(z2 + b2v);
      const bool on = k < K && n < N;
      const float err = on ? y - tv[rt] : 0.0f;
      sq = fmaf(err, err, sq);
      const float d2 = dscale * err * y * (1.0f - y);
      gb2 += d2;
      return d2;
    };
    // the gradients of NR (1 or 2) consecutive row tiles from r0
    auto tiles = [&](auto r0_c, auto nr_c) {
      constexpr int r0 = decltype(r0_c)::value, NR = decltype(nr_c)::value;
      float d2[NR];
      d2[0] = delta2(std::integral_constant<int, r0>{});
      if constexpr (NR == 2) d2[NR - 1] = delta2(std::integral_constant<int, r0 + 1>{});
      float av[NR][4], sl[NR][4];
#pragma unroll
      for (int j = 0; j < NR; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) av[j][i] = sigmoid_slope(zz[r0 + j][i], sl[j][i]);
        Dd[j * 64 + l16 * 4 + lg] = d2[j];
        *reinterpret_cast<f32x4_s *>(Dst + j * 256 + l16 * 16 + 4 * lg) = f32x4_s{av[j][0], av[j][1], av[j][2], av[j][3]};
      }
      // gW2^T += a^T delta2 (M = hidden, N = outputs, K = the tile's rows)
#pragma unroll
      for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float dv = Dd[j * 64 + (4 * s + lg) * 4 + (l16 & 3)];
          g2 = __builtin_amdgcn_mfma_f32_16x16x4f32(Dst[j * 256 + (4 * s + lg) * 16 + l16], l16 < 4 ? dv : 0.0f,
                                                   g2, 0, 0, 0);
        }
      // delta1^T = W2^T delta2^T (the pre-update W2), times the slope
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const f32x4_s bp = __builtin_amdgcn_mfma_f32_16x16x4f32(W2s[lg * HP + h0 + l16], d2[j],
                                                               f32x4_s{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        *reinterpret_cast<f32x4_s *>(Dst + j * 256 + l16 * 16 + 4 * lg) =
            f32x4_s{bp[0] * sl[j][0], bp[1] * sl[j][1], bp[2] * sl[j][2], bp[3] * sl[j][3]};
      }
      // gW1 += delta1^T [X 1] (M = hidden, N = features, K = the tile's rows)
#pragma unroll
      for (int ft = 0; ft < 4; ++ft) {
        if (ft < FT) {
          f32x4_s g = gacc[ft];
#pragma unroll
          for (int j = 0; j < NR; ++j) {
            const float *da = Dst + j * 256 + lg * 16 + l16;
            const float *xb = Xs + ((r0 + j) * 16 + lg) * XS + ft * 16 + l16;
#pragma unroll
            for (int s = 0; s < 4; ++s) g = __builtin_amdgcn_mfma_f32_16x16x4f32(da[s * 64], xb[s * 4 * XS], g, 0, 0, 0);
          }
          gacc[ft] = g;
        }
      }
    };
    auto pair_b = [&](auto r0_c) {
      constexpr int r0 = decltype(r0_c)::value;
      if (r0 + 1 < NPT) tiles(r0_c, std::integral_constant<int, 2>{});
      else if (r0 < NPT) tiles(r0_c, std::integral_constant<int, 1>{});
    };
    pair_b(std::integral_constant<int, 0>{});
    pair_b(std::integral_constant<int, 2>{});
    pair_b(std::integral_constant<int, 4>{});
    pair_b(std::integral_constant<int, 6>{});
    if (wave == 0 && loss_hist) {
      const float sqw = wave_sum(sq);
      if (lane == 0) loss_hist[(int64_t)blockIdx.x * epochs + e] = sqw * inv_nk;
    }
    // ======================= update: this wave's W1 rows and W2 columns, b2
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) {
      if (ft < FT) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int h = h0 + 4 * lg + i, d = 16 * ft + l16;
          if (h < H && d < D1) {
            const int o = h * XS + d;
            float wv = W1s[o];
            gd_update(wv, c1[ft][i], lr, gacc[ft][i], compensated);
            W1s[o] = wv;
          }
        }
      }
    }
    if (l16 < K) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int h = h0 + 4 * lg + i;
        if (h < H) {
          const int o = l16 * HP + h;
          float wv = W2s[o];
          gd_update(wv, c2[i], lr, g2[i], compensated);
          W2s[o] = wv;
        }
      }
    }
    // every lane of group lg holds the row sum of output lg after sum16
    gb2 = sum16(gb2);
    if (lg < K) gd_update(b2v, cb, lr, gb2, compensated);
  }
  __syncthreads();

  // ---- write the trained parameters (and compensation) back once
  if (own) {
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) {
      if (ft < FT) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int h = h0 + 4 * lg + i, d = 16 * ft + l16;
          if (h < H && d < D1) {
            const int o = d < D ? h * D + d : oB1 + h;
            P[o] = W1s[h * XS + d];
            if (compensated) Cp[o] = c1[ft][i];
          }
        }
      }
    }
    if (l16 < K) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int h = h0 + 4 * lg + i;
        if (h < H) {
          P[oW2 + l16 * H + h] = W2s[l16 * HP + h];
          if (compensated) Cp[oW2 + l16 * H + h] = c2[i];
        }
      }
    }
  }
  if (wave == 0 && l16 == 0 && lg < K) {
    P[oB2 + lg] = b2v;
    if (compensated) Cp[oB2 + lg] = cb;
  }
}

template <int NW, int KO>
hipError_t launch_hsplit_one(const mlp_batch_item *items, mlp_batch_item one, int n_nets, int n_in, int n_out,
                             size_t lds, const float *X, const float *T, float *theta, float *comp, int epochs,
                             float *loss_hist, hipStream_t s) {
  auto kern = k_small_hsplit<NW, KO>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n_nets), dim3(NW * 64), lds, s, items, one, n_in, n_out, X, T, theta, comp,
                     epochs, loss_hist);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_hsplit_nw(const mlp_batch_item *items, mlp_batch_item one, int n_nets, int n_in, int n_out,
                            size_t lds, const float *X, const float *T, float *theta, float *comp, int epochs,
                            float *loss_hist, hipStream_t s) {
  if (n_out <= 3)
    return launch_hsplit_one<NW, 3>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, s);
  return launch_hsplit_one<NW, 4>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs, loss_hist, s);
}

}  // namespace mlpk

namespace mlph {

size_t small_lds_bytes(int n_rows, int n_hidden, int n_in, int threads, bool momentum) {
  mlpk::SmallLayout L(n_rows, n_hidden, n_in, 4, threads / 64);
  return sizeof(float) * (size_t)L.total(momentum);
}

int small_threads(int n_nets, int hint) {
  if (hint == kHiddenSplit || hint == 128 || hint == 256 || hint == 512) return hint;
  return n_nets <= 64 ? 512 : 128;
}

size_t small_launch_lds_bytes(int max_rows, int max_hidden, int n_in, int threads, bool momentum) {
  // the layout grows monotonically with N and H
  return small_lds_bytes(max_rows, max_hidden, n_in, threads, momentum);
}

hipError_t launch_small_train(const mlp_batch_item *items, mlp_batch_item one, int n_nets,
                              int n_in, int n_out, int max_rows, int max_hidden, const float *X,
                              const float *T, float *theta, float *comp, int epochs,
                              float *loss_hist, int act, float mu, float *vel, int threads, hipStream_t s) {
  const mlpk::SmallVariant var{act, mu, vel};
  const bool mom = vel != nullptr;
  if (threads == kHiddenSplit) {
    if (act == 0 && !mom) {
      // one wave per 16 hidden units of the launch's widest net
      const int tiles = (max_hidden + 15) / 16;
      const int nw = tiles <= 1 ? 1 : (tiles <= 2 ? 2 : 4);
      const size_t lds =
          sizeof(float) * (size_t)mlpk::HSplitLayout(max_rows, max_hidden, n_in, nw, n_out <= 3 ? 3 : 4).total();
      if (nw == 1)
        return mlpk::launch_hsplit_nw<1>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs,
                                         loss_hist, s);
      if (nw == 2)
        return mlpk::launch_hsplit_nw<2>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs,
                                         loss_hist, s);
      return mlpk::launch_hsplit_nw<4>(items, one, n_nets, n_in, n_out, lds, X, T, theta, comp, epochs,
                                       loss_hist, s);
    }
    threads = 128;   // the variants run on the row-split form
  }
  // fewer waves when the per-wave partial buffers would not fit in LDS
  while (threads > 128 && small_launch_lds_bytes(max_rows, max_hidden, n_in, threads, mom) > 160 * 1024)
    threads /= 2;
  const size_t lds = small_launch_lds_bytes(max_rows, max_hidden, n_in, threads, mom);
  if (act == 1) {
    // the tanh variant is instantiated for 8 waves only; the host API
    // checks that its LDS plan fits before launching
    if (threads != 512) return hipErrorInvalidValue;
    return mlpk::launch_nw<8, 1>(max_hidden, items, one, n_nets, n_in, n_out, lds, X, T, theta, comp,
                                 epochs, loss_hist, var, s);
  }
  if (threads == 512)
    return mlpk::launch_nw<8, 0>(max_hidden, items, one, n_nets, n_in, n_out, lds, X, T, theta, comp,
                                 epochs, loss_hist, var, s);
  if (threads == 256)
    return mlpk::launch_nw<4, 0>(max_hidden, items, one, n_nets, n_in, n_out, lds, X, T, theta, comp,
                                 epochs, loss_hist, var, s);
  return mlpk::launch_nw<2, 0>(max_hidden, items, one, n_nets, n_in, n_out, lds, X, T, theta, comp,
                               epochs, loss_hist, var, s);
}

}  // namespace mlph
