// Large-N minibatch trainer: one persistent, cooperatively launched kernel
// runs every minibatch step of every epoch (arxiv 1908.07847, section 2.2:
// feed forward, error, backpropagation, gradient-descent update; contiguous
// minibatches in stored order).
//
// Work of one step (minibatch of m <= b rows) is split over a Gi x Gj grid
// of workgroups: workgroup (i, j) owns row block i (RB = b / Gi rows) and
// hidden block j (HB = Hp / Gj units, at most 256).  The block's 16-unit
// hidden tiles are dealt round-robin to the workgroup's 8 waves (two per
// SIMD, so one wave's matrix-core work overlaps the other's vector work).  The
// two large contractions run on MFMA:
//   z1 = X W1^T           M = rows,   N = hidden,   K = features
//   gW1 = delta1^T X      M = hidden, N = features, K = rows
// in float32 (v_mfma_f32_16x16x4_f32), bf16 or OCP e4m3 (16x16x32, float32
// accumulation).  Everything else -- biases, sigmoid, the K-output layer,
// the deltas, gb1, gW2, gb2, the loss and the update of the float32 master
// parameters -- is float32 VALU work.
//
// A step is three phases separated by grid barriers:
//   1  each workgroup forms a = sigma(z1 + b1) for its tile, row chunk by row
//      chunk, and the partial output pre-activation over its hidden block;
//      the Gj partials of a row meet in the workspace (skipped when Gj = 1).
//   2  each workgroup completes z2, y, delta2 (and the loss) for its rows,
//      recomputes its tile of a (cheaper on MFMA than a trip through HBM),
//      forms delta1 = (delta2 W2) . a (1 - a) with the pre-update W2, and
//      accumulates its partial gW1, gb1, gW2 (and gb2) over its rows.
//   3  every workgroup sums a slice of the Gi partials of each parameter in
//      a fixed order and applies the (optionally Kahan-compensated) update.
// All reductions use fixed orders, so runs are bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "mlp_device.hpp"
#include "mlp_large.hpp"

namespace mlpk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxNW = 8;    // most waves per workgroup (the LDS plan is sized for it)
constexpr int kProbeLT = 256;  // threads per workgroup of the barrier probe
constexpr int kRC = 32;      // rows per chunk
constexpr int kMaxD = 64;    // features
constexpr int kMaxK = 4;     // outputs
constexpr int kMaxNets = 64; // nets sharing X in one launch

struct LargeArgs {
  const float *X, *T;
  float *theta, *comp, *loss_hist;
  float *z2p;        // [M Gj][b][4] partial output pre-activations
  float *gp;         // [Gi][M P] partial gradients
  float *lossp;      // [Gi][M] partial squared errors
  float *amax;       // [2][G] W1 amax partials, [2][G] delta1 amax partials, [G] |X|
  float *acc;        // [M]: epoch loss accumulators
  unsigned short *w1h;  // [P] bf16 copy of theta written by each update (bf16 operands, one net), else null
  unsigned *bar;     // grid-barrier counters and status words (see GridSync)
  uint64_t wait_limit;  // wall-clock ticks a grid-barrier wait may take
  int64_t N, b;
  int D, H, Hp, K, Gi, Gj, M, RBP, epochs, steps_per_epoch;
  float lr[kMaxNets];  // learning rate of each net
};

// ---------------------------------------------------------------- barrier
// Hierarchical grid barrier.  Every workgroup is resident (cooperative
// launch).  Arrivals are counted per XCD (the physical XCC id, read from the
// hardware register); the last arriver of an XCD makes that XCD's L2
// contents visible device-wide (one agent-scope release per XCD instead of
// one per workgroup) and bumps the global count; everyone waits for the
// global count and then acquires.  Counters only grow: the k-th barrier waits
// for k arrivals per member.
//
// Every wait is bounded in time: a wait that is still unsatisfied after
// `limit` ticks of the constant-rate wall clock sets the sticky give-up word
// and returns false, and every other wait returns false as soon as it sees
// that word.  The trainer then leaves its step loop in every workgroup (no
// workgroup waits on one that has left), so a grid that cannot complete a
// barrier ends with an error the host can read instead of hanging.
//
// Counter block (unsigned, 16 apart so each sits on its own 64-byte line),
// at the head of the workspace:
//   [0] XCD-leader arrivals, [16] give-up word (the status the host reads),
//   [16*(2+x)] arrivals on XCD x, [16*(10+x)] members on XCD x,
//   [16*18] registrations, [16*19] non-finite word (finite check).
constexpr int kBarWords = 16 * 20;
constexpr int kGiveUpWord = 16;
constexpr int kNonFiniteWord = 16 * 19;

__device__ __forceinline__ unsigned xcc_id() {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;  // HW_REG_XCC_ID[3:0]
#else
  return 0;
#endif
}

struct GridSync {
  unsigned *bar;
  unsigned x, members, n_xcd, k;
  uint64_t limit;  // wall-clock ticks one wait may take
  __device__ bool spin(unsigned *ctr, unsigned target) {
    // the clock is first read at the first check (64 spins in), off the
    // path of a barrier that completes quickly
    uint64_t t0 = 0;
    bool timing = false;
    unsigned spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 63u) == 0 || limit == 0) {
        if (__hip_atomic_load(bar + kGiveUpWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        const uint64_t now = wall_clock64();
        if (!timing) {
          t0 = now;
          timing = true;
        }
        if (now - t0 >= limit) {
          __hip_atomic_store(bar + kGiveUpWord, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return false;
        }
      }
    }
    return true;
  }
  // every workgroup registers its XCD once (thread 0 only); false: gave up
  __device__ bool init(unsigned *b, unsigned G, uint64_t wait_limit) {
    bar = b;
    limit = wait_limit;
    x = xcc_id();
    k = 0;
    __hip_atomic_fetch_add(bar + 16 * (10 + x), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(bar + 16 * 18, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = spin(bar + 16 * 18, G);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    members = __hip_atomic_load(bar + 16 * (10 + x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    n_xcd = 0;
    for (int q = 0; q < 8; ++q)
      n_xcd += __hip_atomic_load(bar + 16 * (10 + q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0u;
    return ok;
  }
  // thread 0 only, between two __syncthreads; false: gave up
  __device__ bool arrive_and_wait() {
    k += 1;
    const unsigned old =
        __hip_atomic_fetch_add(bar + 16 * (2 + x), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == k * members) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const bool ok = spin(bar, k * n_xcd);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
  }
};

// ---------------------------------------------------------------- operands
// OCP e4m3 with a power-of-two scale 2^e: saturate to +-448 first (the
// hardware conversion would give NaN above 448), round to nearest even.
__device__ __forceinline__ uint32_t pack_e4m3x4(float a, float b, float c, float d) {
  a = fminf(fmaxf(a, -448.f), 448.f);
  b = fminf(fmaxf(b, -448.f), 448.f);
  c = fminf(fmaxf(c, -448.f), 448.f);
  d = fminf(fmaxf(d, -448.f), 448.f);
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, v, true);
  return (uint32_t)v;
}

// e such that amax * 2^e <= 448 < amax * 2^(e+1) (0 for amax == 0).
__device__ __forceinline__ int e4m3_scale_exp(float amax) {
  if (!(amax > 0.0f)) return 0;
  int ex;
  float f = frexpf(amax, &ex);  // amax = f * 2^ex, f in [0.5, 1); 448 = 0.875 * 2^9
  return (f <= 0.875f) ? 9 - ex : 8 - ex;
}

// One e4m3 byte (saturated, round to nearest even).
__device__ __forceinline__ uint8_t e4m3_byte(float v) {
  v = fminf(fmaxf(v, -448.f), 448.f);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xff);
}

// Hidden-layer sigmoid of the reduced-precision forms: the hardware base-2
// exponential of t = -z log2(e), rounded once, and the hardware reciprocal.
// The rounding of t scales e^-z by 2^(|t| 2^-24), so e^-z is good to about
// |z| 7e-8 relative (1e-6 at |z| = 15) and sigma to that times (1 - sigma)
// plus a few float ulps.  The contraction operands of these forms carry
// 2^-9 (bf16) or 2^-4 (e4m3) relative rounding; the float32 form keeps the
// compensated evaluation of sigmoid_e.  PREC selects the form by operand type.
template <int PREC>
__device__ __forceinline__ float hidden_sigmoid_e(float z, float &e_out) {
  if (PREC == 0) return sigmoid_e(z, e_out);
  const float t = fminf(-z * 1.44269502162933349609375f, 126.0f);
  const float e = __builtin_amdgcn_exp2f(t);
  e_out = e;
  return __builtin_amdgcn_rcpf(1.0f + e);
}
template <int PREC>
__device__ __forceinline__ float hidden_sigmoid(float z) {
  float e;
  return hidden_sigmoid_e<PREC>(z, e);
}
// sigma and its slope e^-z sigma^2 (see sigmoid_slope)
template <int PREC>
__device__ __forceinline__ float hidden_sigmoid_slope(float z, float &slope) {
  float e;
  const float a = hidden_sigmoid_e<PREC>(z, e);
  slope = (e * a) * a;
  return a;
}

constexpr int kStageU = 16;  // loads in flight per thread while staging
constexpr int kPre = 32;     // X elements per thread loaded in one batch for a step's first piece
constexpr int kRedU = 32;    // partial-gradient loads in flight per thread
constexpr int kUpdU = 4;     // parameters per thread per batch when there are at most 4 partials

// q / D for 0 <= q < 2^16 and 1 <= D <= 64 with md = ceil(2^22 / D): the
// error md*D - 2^22 <= D - 1 keeps q*md / 2^22 below the next integer.
__device__ __forceinline__ int div_by(int q, uint32_t md) {
  return (int)(((uint64_t)(uint32_t)q * md) >> 22);
}

// *p if ok, else 0, with the load itself unconditional (it reads *safe
// when !ok): a predicated load becomes a branch around it, and the compiler
// then waits for the load inside that branch, which serialises a batch of
// loads that should be in flight together.
__device__ __forceinline__ float load_if(const float *p, const float *safe, bool ok) {
  const float v = *(ok ? p : safe);
  return ok ? v : 0.0f;
}

// Copy n contiguous floats src[0..n) through registers: each thread loads
// U elements (stride LT, the workgroup's thread count) before storing any,
// so a batch costs one memory round trip.  store(q, v) places element q.
template <int U, int LT, typename F>
__device__ __forceinline__ void stage_flat(const float *src, int n, int tid, F &&store) {
  for (int base = 0; base < n; base += U * LT) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = base + u * LT + tid;
      v[u] = load_if(src + q, src, q < n);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = base + u * LT + tid;
      if (q < n) store(q, v[u]);
    }
  }
}

template <int PREC>
struct Ops;

// float32: operands are floats, one per lane per 16x16x4 step.
template <>
struct Ops<0> {
  static constexpr int KSTEP = 4;
  typedef float elem;
  static constexpr int XROW = 66;   // LDS row stride (floats) of X rows and W1 rows
};
// bf16 / e4m3: 8 operands per lane per 16x16x32 step.
template <>
struct Ops<1> {
  static constexpr int KSTEP = 32;
  typedef __bf16 elem;
  static constexpr int XROW = 72;   // bf16 elements per X / W1 row (64 + pad)
  static constexpr int XTP = 8;     // pad of a transposed X row (RB rows + pad)
};
template <>
struct Ops<2> {
  static constexpr int KSTEP = 32;
  typedef uint8_t elem;
  static constexpr int XROW = 80;   // bytes per X / W1 row (64 + pad)
  static constexpr int XTP = 16;
};

// LDS plan (bytes), shared by host and device.
template <int PREC>
struct LLayout {
  int HB, RB;
  __host__ __device__ LLayout(int hb, int rb) : HB(hb), RB(rb) {}
  static constexpr int esz = sizeof(typename Ops<PREC>::elem);
  __host__ __device__ int xr() const { return 0; }
  // the whole row block is staged once per step: X rows (and, for the 8-wide
  // operand formats, X transposed so that 8 consecutive rows are contiguous)
  __host__ __device__ int xts() const { return RB + (PREC == 0 ? 0 : Ops<(PREC == 0 ? 1 : PREC)>::XTP); }
  __host__ __device__ int xt() const { return xr() + RB * Ops<PREC>::XROW * esz; }
  __host__ __device__ int w1() const { return xt() + (PREC == 0 ? 0 : kMaxD * xts() * esz); }
  __host__ __device__ int b1() const { return w1() + HB * Ops<PREC>::XROW * esz; }
  __host__ __device__ int w2() const { return b1() + HB * 4; }
  __host__ __device__ int d2() const { return w2() + kMaxK * HB * 4; }
  __host__ __device__ int z2w() const { return d2() + RB * 16; }
  __host__ __device__ int red() const { return z2w() + 2 * kMaxNW * kRC * 16; }   // two chunk buffers
  __host__ __device__ int total() const { return red() + 64 * 4; }
};

// KO: outputs the loops run over (K <= KO <= kMaxK; 3 for the usual K = 3).
// NW: waves per workgroup, 4 (one per SIMD) or 8 (two per SIMD, so one
// wave's matrix-core work overlaps the other's vector work).  NHM: hidden
// tiles a wave owns at most, 16 / NW for hidden blocks of up to 256 units,
// or 1 for blocks of at most NW tiles (the loops over a wave's tiles then
// hold one tile: a step's code is far smaller, and fits the instruction
// cache that two CUs share, which the general instance's does not).
template <int PREC, int KO, int NW, int NHM>
__global__ __launch_bounds__(64 * NW, 1) void k_large_train(LargeArgs a) {
  static_assert(NHM >= 1 && NHM <= 16 / NW, "tiles per wave");
  constexpr int kNW = NW, kLT = 64 * NW;
  using O = Ops<PREC>;
  using E = typename O::elem;
  constexpr int XROW = O::XROW;

  // the wave index is uniform over the wave: held in a scalar register, so
  // everything derived from it (tiles, row sets, partial ranges) is too
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // Column blocks: M nets x Gj hidden blocks each (M > 1: nets that share X).
  const int Gc = a.M * a.Gj, G = a.Gi * Gc;
  // XCD-aware placement: workgroups are dispatched round-robin over the 8
  // XCDs, so the Gc workgroups that share a row block (and its X rows) get
  // the same blockIdx % 8 and hence the same L2.
  const int bid = blockIdx.x;
  int gi, gc;
  if (G % 8 == 0 && a.Gi % 8 == 0) {
    const int xcd = bid & 7, q = bid >> 3;
    gc = q % Gc;
    gi = (q / Gc) * 8 + xcd;
  } else {
    gi = bid / Gc;
    gc = bid - gi * Gc;
  }
  const int net = gc / a.Gj, gj = gc - net * a.Gj;
  const int D = a.D, H = a.H, K = a.K;
  // hidden tiles of the block: tile t (units 16 t .. 16 t + 15) belongs to
  // wave t % kNW as its local tile t / kNW; this wave owns NHB of them
  const int HB = a.Hp / a.Gj, NT = HB / 16, NHB = (NT - wave + kNW - 1) / kNW;
  const int RB = (int)(a.b / a.Gi);     // rows of this workgroup's block
  const int RBP = a.RBP;                // rows staged in LDS at a time (divides RB)
  const int NPc = RB / RBP;             // pieces of the block
  // first unit (within the block) of this wave's local tile hb
  auto tile_unit = [&](int hb) { return (hb * kNW + wave) * 16; };
  const int64_t P = (int64_t)D * H + H + (int64_t)H * K + K;
  const int64_t PT = P * a.M;           // parameters of all nets
  const int64_t oB1 = (int64_t)D * H, oW2 = oB1 + H, oB2 = oW2 + (int64_t)H * K;
  float *th = a.theta + (int64_t)net * P;   // this workgroup's net
  const LLayout<PREC> L(HB, RBP);
  const int KS = O::KSTEP;
  const int DK = (D + KS - 1) / KS * KS;      // padded contraction length of z1
  const int NFB = (D + 15) / 16;              // 16-wide feature blocks of gW1
  const int l16 = lane & 15, lg = lane >> 4;  // MFMA lane coordinates

  extern __shared__ float4 smem4[];
  char *smb = reinterpret_cast<char *>(smem4);
  E *xr = reinterpret_cast<E *>(smb + L.xr());
  E *xt = reinterpret_cast<E *>(smb + L.xt());
  E *w1s = reinterpret_cast<E *>(smb + L.w1());
  float *b1s = reinterpret_cast<float *>(smb + L.b1());
  float *w2s = reinterpret_cast<float *>(smb + L.w2());
  float *d2s = reinterpret_cast<float *>(smb + L.d2());
  float *z2w = reinterpret_cast<float *>(smb + L.z2w());
  float *red = reinterpret_cast<float *>(smb + L.red());
  // Workgroup max / sum of one value per wave (lane 0's), through
  // red[slot .. slot + 7], in a fixed order; every thread gets the result.
  auto wg_reduce_max = [&](float v, int slot) {
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    if (lane == 0) red[slot + wave] = v;
    __syncthreads();
    float m = red[slot];
#pragma unroll
    for (int w = 1; w < kNW; ++w) m = fmaxf(m, red[slot + w]);
    return m;
  };
  auto wg_reduce_sum = [&](float v, int slot) {
    v = wave_sum(v);
    if (lane == 0) red[slot + wave] = v;
    __syncthreads();
    float t[kNW];
#pragma unroll
    for (int w = 0; w < kNW; ++w) t[w] = red[slot + w];
#pragma unroll
    for (int st = 1; st < kNW; st *= 2)
#pragma unroll
      for (int w = 0; w < kNW; w += 2 * st) t[w] += t[w + st];
    return t[0];
  };

  // ok_s: 0 once a grid-barrier wait of this workgroup has given up
  __shared__ int ok_s;
  GridSync gs;
  if (tid == 0) ok_s = gs.init(a.bar, (unsigned)G, a.wait_limit) ? 1 : 0;
  __syncthreads();
  bool ok = ok_s != 0;
  // false when the barrier gave up (uniform over the workgroup)
  auto barrier = [&]() -> bool {
    __syncthreads();  // this workgroup's stores are complete (in L2) before it arrives
    if (tid == 0 && !gs.arrive_and_wait()) ok_s = 0;
    __syncthreads();
    return ok_s != 0;
  };

  // ---- one-time: dataset amax of |X| for the e4m3 X scale
  int ex = 0;
  if (PREC == 2 && ok) {
    float m = 0.0f;
    const int64_t nx = a.N * D;
    for (int64_t q = (int64_t)bid * kLT + tid; q < nx; q += (int64_t)G * kLT) m = fmaxf(m, fabsf(a.X[q]));
    m = wg_reduce_max(m, 0);
    if (tid == 0) a.amax[4 * G + bid] = m;
    ok = barrier();
    float mm = 0.0f;
    for (int g = 0; g < G; ++g) mm = fmaxf(mm, a.amax[4 * G + g]);
    ex = e4m3_scale_exp(mm);
  }
  const float sx = ldexpf(1.0f, ex), isx = ldexpf(1.0f, -ex);

  // ---- X staging.  A piece of a step's row block (RBP rows) is a
  // contiguous run of X (RBP x D floats); rows past the end of a short last
  // minibatch are zero.  Piece 0 of a step is staged at the start of the
  // step, its first kPre * kLT elements through registers all loaded before
  // the first store; other pieces are staged in batches of kStageU.
  const int XTS = L.xts();
  const uint32_t mdD = ((1u << 22) + (uint32_t)D - 1) / (uint32_t)D;
  auto block_rows = [&](int st, int pc, int64_t &rb0_, int &rows_) {
    const int sidx_ = st % a.steps_per_epoch;
    const int64_t r0_ = (int64_t)sidx_ * a.b;
    const int64_t m_ = min((int64_t)a.b, a.N - r0_);
    const int64_t first = (int64_t)gi * RB + (int64_t)pc * RBP;   // within the minibatch
    rb0_ = r0_ + first;
    rows_ = (int)max((int64_t)0, min((int64_t)RBP, m_ - first));
  };
  // A staging unit is 8 consecutive rows of one feature: unit u holds rows
  // 8 (u / D) .. +7 and feature u % D.  Lanes run over features, so each of
  // the unit's 8 loads is a coalesced run of an X row; the 8 values land in
  // the row-major copy one by one and in the transposed copy (operand of
  // gW1 = delta1^T X) as one 16-byte (bf16) or 8-byte (e4m3) store.
  constexpr int kUnitsPre = kPre / 8;      // units per thread held in xpre
  constexpr int kUnitsBatch = kStageU / 8;  // units per thread per direct batch
  const int n_units = RBP / 8 * D;
  auto put_unit = [&](int u, const float *v) {
    const int r8 = div_by(u, mdD), c = u - r8 * D, rr = r8 * 8;
    if (PREC == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) reinterpret_cast<float *>(xr)[(rr + j) * XROW + c] = v[j];
    } else if (PREC == 1) {
      bf16x8 t;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        t[j] = (__bf16)v[j];
        reinterpret_cast<__bf16 *>(xr)[(rr + j) * XROW + c] = t[j];
      }
      *reinterpret_cast<bf16x8 *>(reinterpret_cast<__bf16 *>(xt) + c * XTS + rr) = t;
    } else {
      uint64_t t = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint8_t bv = e4m3_byte(v[j] * sx);
        reinterpret_cast<uint8_t *>(xr)[(rr + j) * XROW + c] = bv;
        t |= (uint64_t)bv << (8 * j);
      }
      *reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(xt) + c * XTS + rr) = t;
    }
  };
  // the 8 values of unit u (zero past the real rows of the piece)
  auto load_unit = [&](const float *src, int rows_, int u, float *v) {
    const int r8 = div_by(u, mdD), c = u - r8 * D, rr = r8 * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = load_if(src + ((rr + j) * D + c), a.X, u < n_units && rr + j < rows_);
  };
  auto load_x = [&](int st, float (&v)[kPre]) {
    int64_t rb0_;
    int rows_;
    block_rows(st, 0, rb0_, rows_);
    const float *src = a.X + rb0_ * D;
    int tid_o = tid;
    asm volatile("" : "+v"(tid_o));   // addresses formed here, per step, not hoisted out of the loop
#pragma unroll
    for (int k = 0; k < kUnitsPre; ++k) load_unit(src, rows_, k * kLT + tid_o, v + 8 * k);
  };
  // stage piece pc of step st; with v (piece 0 only) its first
  // kUnitsPre * kLT units come from the registers
  auto store_x = [&](int st, int pc, const float (*v)[kPre]) {
    int from = 0;
    if (v) {
#pragma unroll
      for (int k = 0; k < kUnitsPre; ++k) {
        const int u = k * kLT + tid;
        if (u < n_units) put_unit(u, *v + 8 * k);
      }
      from = kUnitsPre * kLT;
    }
    if (n_units > from) {
      int64_t rb0_;
      int rows_;
      block_rows(st, pc, rb0_, rows_);
      const float *src = a.X + rb0_ * D;
      for (int base = from; base < n_units; base += kUnitsBatch * kLT) {
        float w[kStageU];
#pragma unroll
        for (int k = 0; k < kUnitsBatch; ++k) load_unit(src, rows_, base + k * kLT + tid, w + 8 * k);
#pragma unroll
        for (int k = 0; k < kUnitsBatch; ++k) {
          const int u = base + k * kLT + tid;
          if (u < n_units) put_unit(u, w + 8 * k);
        }
      }
    }
  };
  float xpre[kPre];

  // LDS operand padding (feature columns D..DK, hidden rows past H) is
  // written once here; the per-step staging writes only real entries.
  for (int q = tid; q < L.b1() / 4; q += kLT) reinterpret_cast<float *>(smb)[q] = 0.0f;
  __syncthreads();

  const int total_steps = a.epochs * a.steps_per_epoch;
  int step = 0;
  for (; ok && step < total_steps; ++step) {
    const int e = step / a.steps_per_epoch, sidx = step - e * a.steps_per_epoch;
    const int64_t r0 = (int64_t)sidx * a.b;
    const int64_t m = min((int64_t)a.b, a.N - r0);      // rows in this minibatch
    const int64_t rb0 = r0 + (int64_t)gi * RB;          // first row of this block
    const int rows_here = (int)max((int64_t)0, min((int64_t)RB, m - (int64_t)gi * RB));
    const float dscale = 2.0f / ((float)m * (float)K);

    // ---- the first piece of this step's row block of X: its loads are
    // issued first, so they are in flight with the W1 slice's (and the e4m3
    // scale partials') and the staging costs one memory round trip, not two
    // (33-256-3, same-box A/B: bf16 6.65 -> 6.43 ms per epoch, e4m3 7.39 ->
    // 7.20; the wide e4m3 form 15.91 -> 15.19; the wide bf16 form, once its
    // W1 slice comes from the bf16 copy, 12.84 -> 12.77; the wide float32
    // form, once its slice is one batch of 16-byte loads, 25.03 -> 24.77).
    // (Loading it during the previous step's update keeps the values live
    // across the partial sums, which every instance spills.)
    //
    // e4m3: the amax partials of the previous update (W1) and of the
    // previous step (delta1), issued ahead of X so the scales' reduction
    // waits for them alone (loaded at every step, without a branch that
    // would make the compiler wait for them before X; used after the first).
    // One workgroup per CU keeps G <= kLT, and a repeated index leaves a
    // maximum unchanged.
    float pw = 0.0f, pd = 0.0f;
    if (PREC == 2) {
      const int g = min(tid, G - 1), par = step & 1;
      pw = a.amax[par * G + g];
      pd = a.amax[2 * G + (par ^ 1) * G + g];
    }
    load_x(step, xpre);

    // ---- scales of this step (e4m3): W1 from the master, delta1 delayed
    int ew = 0, ed = 0;
    if (PREC == 2) {
      const int par = step & 1;
      if (step == 0) {
        float mw = 0.0f;
        for (int64_t q = tid; q < (int64_t)H * D; q += kLT) mw = fmaxf(mw, fabsf(th[q]));
        ew = e4m3_scale_exp(wg_reduce_max(mw, 0));
        __syncthreads();
        // first step: the bound max_h sum_k |W2[k][h]| / (8 m K), in float32, left to right
        float bound = 0.0f;
        for (int h = 0; h < H; ++h) {
          float col = 0.0f;
          for (int k = 0; k < K; ++k) col = col + fabsf(th[oW2 + (int64_t)k * H + h]);
          if (col > bound) bound = col;
        }
        bound = bound / (float)(8 * m * K);
        ed = e4m3_scale_exp(bound);
      } else {
        for (int g = tid + kLT; g < G; g += kLT) {
          pw = fmaxf(pw, a.amax[par * G + g]);
          pd = fmaxf(pd, a.amax[2 * G + (par ^ 1) * G + g]);
        }
        ew = e4m3_scale_exp(wg_reduce_max(pw, 24));
        ed = e4m3_scale_exp(wg_reduce_max(pd, 32));
      }
    }
    const float sw = ldexpf(1.0f, ew), isw = ldexpf(1.0f, -ew);
    const float sd = ldexpf(1.0f, ed), isd = ldexpf(1.0f, -ed);

    // ---- stage this workgroup's slice of W1 (operand precision), b1, W2.
    // The slice is a contiguous run of theta; every thread issues all of its
    // loads before the first store (one memory round trip, not one per row).
    {
      // b1 and W2 of the hidden block: (1 + kMaxK) HB <= 5 kLT values,
      // loaded together with the first batch of W1
      constexpr int kBW = ((1 + kMaxK) * 256 + kLT - 1) / kLT;
      float bw[kBW];
#pragma unroll
      for (int u = 0; u < kBW; ++u) {
        const int q = tid + u * kLT;             // q < HB: b1, else W2 row k = q / HB - 1
        const int k = q / HB - 1, hl = q - (k + 1) * HB, h = gj * HB + hl;
        const bool ok = q < (1 + kMaxK) * HB && h < H && k < K;
        bw[u] = load_if(th + (k < 0 ? oB1 + h : oW2 + (int64_t)k * H + h), th, ok);
      }
      const int hv = max(0, min(HB, H - gj * HB));          // real hidden units here
      if (PREC == 1 && a.w1h != nullptr && step > 0) {
        // bf16, one net, after the first step of the launch: the slice of
        // the bf16 copy of W1 that the previous update wrote (the rounding
        // below, done once per parameter instead of once per workgroup):
        // half the bytes, and with D a multiple of 8 eight values per
        // 16-byte load, so the whole slice is one batch of loads
        const unsigned short *hsrc = a.w1h + (int64_t)gj * HB * D;
        const int n = hv * D;
        int tid_o = tid;
        asm volatile("" : "+v"(tid_o));   // addresses formed per step (see the X staging)
        if ((D & 7) == 0) {
          constexpr int kV = 4;   // a 256 x 64 slice on 8 waves, a 128 x 64 one on 4
          for (int base = 0; base < n; base += 8 * kV * kLT) {
            uint4 v[kV];
#pragma unroll
            for (int u = 0; u < kV; ++u) {
              const int q = base + 8 * (u * kLT + tid_o);
              v[u] = *reinterpret_cast<const uint4 *>(hsrc + (q < n ? q : 0));
            }
#pragma unroll
            for (int u = 0; u < kV; ++u) {
              const int q = base + 8 * (u * kLT + tid_o);
              if (q < n) {
                const int hl = div_by(q, mdD), c = q - hl * D;   // the 8 values share row hl
                *reinterpret_cast<uint4 *>(reinterpret_cast<unsigned short *>(w1s) + hl * XROW + c) = v[u];
              }
            }
          }
        } else {
          for (int base = 0; base < n; base += kStageU * kLT) {
            unsigned short v[kStageU];
#pragma unroll
            for (int u = 0; u < kStageU; ++u) {
              const int q = base + u * kLT + tid_o;
              v[u] = hsrc[q < n ? q : 0];
            }
#pragma unroll
            for (int u = 0; u < kStageU; ++u) {
              const int q = base + u * kLT + tid_o;
              if (q < n) {
                const int hl = div_by(q, mdD), c = q - hl * D;
                reinterpret_cast<unsigned short *>(w1s)[hl * XROW + c] = v[u];
              }
            }
          }
        }
      } else if (PREC == 0 && (D & 3) == 0 && (reinterpret_cast<uintptr_t>(th) & 15) == 0) {
        // float32 with D a multiple of 4 (and theta 16-byte aligned): four
        // values (of one row) per 16-byte load, the whole slice in one batch
        // of at most eight loads per thread (a 256 x 64 slice on 8 waves),
        // and two 8-byte LDS stores
        const float *w1src = th + (int64_t)gj * HB * D;
        const int n = hv * D;
        int tid_o = tid;
        asm volatile("" : "+v"(tid_o));   // addresses formed per step (see the X staging)
        constexpr int kV = 8;
        for (int base = 0; base < n; base += 4 * kV * kLT) {
          float4 v[kV];
#pragma unroll
          for (int u = 0; u < kV; ++u) {
            const int q = base + 4 * (u * kLT + tid_o);
            v[u] = *reinterpret_cast<const float4 *>(w1src + (q < n ? q : 0));
          }
#pragma unroll
          for (int u = 0; u < kV; ++u) {
            const int q = base + 4 * (u * kLT + tid_o);
            if (q < n) {
              const int hl = div_by(q, mdD), c = q - hl * D;
              float2 *d = reinterpret_cast<float2 *>(reinterpret_cast<float *>(w1s) + hl * XROW + c);
              d[0] = float2{v[u].x, v[u].y};
              d[1] = float2{v[u].z, v[u].w};
            }
          }
        }
      } else {
        const float *w1src = th + (int64_t)gj * HB * D;
        stage_flat<kStageU, kLT>(w1src, hv * D, tid, [&](int q, float v) {
          const int hl = div_by(q, mdD), c = q - hl * D;
          const int o = hl * XROW + c;
          if (PREC == 0) reinterpret_cast<float *>(w1s)[o] = v;
          if (PREC == 1) reinterpret_cast<__bf16 *>(w1s)[o] = (__bf16)v;
          if (PREC == 2) reinterpret_cast<uint8_t *>(w1s)[o] = e4m3_byte(v * sw);
        });
      }
#pragma unroll
      for (int u = 0; u < kBW; ++u) {
        const int q = tid + u * kLT;
        if (q < HB) b1s[q] = bw[u];
        else if (q < (1 + kMaxK) * HB) w2s[q - HB] = bw[u];
      }
    }
    // ---- this step's row block of X (its first piece), loaded at the start
    // of the step (see there) and stored after the W1 slice.
    store_x(step, 0, &xpre);
    int cur_piece = 0;   // piece of the row block held in LDS
    auto stage_piece = [&](int pc) {
      if (pc == cur_piece) return;
      __syncthreads();   // every wave is done with the previous piece
      store_x(step, pc, nullptr);
      cur_piece = pc;
      __syncthreads();
    };
    __syncthreads();

    // z1 tiles for rows [c0, c0 + 32) of the block and every hidden block hb
    // of this wave: zt[hb][rs] holds rows c0 + 16 rs + 4 lg + i, hidden unit
    // 16 hb + l16.  The X operands of the 32 rows are loaded once and reused
    // across hidden blocks; all MFMAs are issued before any result is used.
    // bf16 / e4m3 W1 operands of this wave's hidden tiles are the same for
    // every row chunk of the step: read them from LDS once, keep them in
    // registers (float32 operands would take 64 registers and stay in LDS)
    bf16x8 w1b[NHM][2];
    long w1e[NHM][2];
    if (PREC != 0) {
#pragma unroll
      for (int hb = 0; hb < NHM; ++hb)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const bool on = hb < NHB;
          const int o = on ? (tile_unit(hb) + l16) * XROW + 8 * lg + 32 * ks : 0;
          if (PREC == 1) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const __bf16 *>(w1s) + o);
            const bf16x8 zero = {};
            w1b[hb][ks] = on ? v : zero;
          } else {
            const long v = *reinterpret_cast<const long *>(reinterpret_cast<const uint8_t *>(w1s) + o);
            w1e[hb][ks] = on ? v : 0l;
          }
        }
    }
    // LDS rows of X and W1 hold kMaxD = 64 columns, those past D zero, so
    // every operand load below reads a valid address and the padding adds
    // exact zeros: the loads need no guard, and the float32 contraction runs
    // in groups of 4 k-steps (16 features), whole groups up to DK.  A tile's
    // operands are loaded together, ahead of its products (one LDS round trip
    // per tile, not one per k-step).
    auto z1_tiles = [&](int c0, f32x4 (&zt)[NHM][2]) {
      if (PREC == 0) {
        float xa[2][16];
#pragma unroll
        for (int rs = 0; rs < 2; ++rs)
#pragma unroll
          for (int st = 0; st < 16; ++st)
            xa[rs][st] = reinterpret_cast<const float *>(xr)[(c0 + rs * 16 + l16) * XROW + lg + 4 * st];
#pragma unroll
        for (int hb = 0; hb < NHM; ++hb) {
          f32x4 z0 = {0.f, 0.f, 0.f, 0.f}, z1v = {0.f, 0.f, 0.f, 0.f};
          if (hb < NHB) {
            const float *wb = reinterpret_cast<const float *>(w1s) + (tile_unit(hb) + l16) * XROW + lg;
            float wv[16];
#pragma unroll
            for (int st = 0; st < 16; ++st) wv[st] = wb[4 * st];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              if (16 * g < DK) {
#pragma unroll
                for (int s = 4 * g; s < 4 * g + 4; ++s) {
                  z0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[0][s], wv[s], z0, 0, 0, 0);
                  z1v = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[1][s], wv[s], z1v, 0, 0, 0);
                }
              }
            }
          }
          zt[hb][0] = z0;
          zt[hb][1] = z1v;
        }
      } else if (PREC == 1) {
        bf16x8 xa[2][2];
#pragma unroll
        for (int rs = 0; rs < 2; ++rs)
#pragma unroll
          for (int ks = 0; ks < 2; ++ks)
            xa[rs][ks] = *reinterpret_cast<const bf16x8 *>(
                reinterpret_cast<const __bf16 *>(xr) + (c0 + rs * 16 + l16) * XROW + 8 * lg + 32 * ks);
#pragma unroll
        for (int hb = 0; hb < NHM; ++hb) {
          f32x4 z0 = {0.f, 0.f, 0.f, 0.f}, z1v = {0.f, 0.f, 0.f, 0.f};
          if (hb < NHB) {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
              z0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[0][ks], w1b[hb][ks], z0, 0, 0, 0);
              z1v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[1][ks], w1b[hb][ks], z1v, 0, 0, 0);
            }
          }
          zt[hb][0] = z0;
          zt[hb][1] = z1v;
        }
      } else {
        long xa[2][2];
#pragma unroll
        for (int rs = 0; rs < 2; ++rs)
#pragma unroll
          for (int ks = 0; ks < 2; ++ks)
            xa[rs][ks] = *reinterpret_cast<const long *>(
                reinterpret_cast<const uint8_t *>(xr) + (c0 + rs * 16 + l16) * XROW + 8 * lg + 32 * ks);
#pragma unroll
        for (int hb = 0; hb < NHM; ++hb) {
          f32x4 z0 = {0.f, 0.f, 0.f, 0.f}, z1v = {0.f, 0.f, 0.f, 0.f};
          if (hb < NHB) {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
              z0 = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xa[0][ks], w1e[hb][ks], z0, 0, 0, 0);
              z1v = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xa[1][ks], w1e[hb][ks], z1v, 0, 0, 0);
            }
          }
          zt[hb][0] = z0 * (isx * isw);
          zt[hb][1] = z1v * (isx * isw);
        }
      }
    };

    // ================================================================ phase 1
    // z2 partial over this workgroup's hidden block for the 32 rows of chunk
    // c0 of the piece in LDS; out(rr, k, v) receives row rr's sum for output k
    auto z2_chunk = [&](int c0, auto &&out) {
      float zp[2][4][KO];
#pragma unroll
      for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < KO; ++k) zp[rs][i][k] = 0.0f;
      f32x4 zt[NHM][2];
      z1_tiles(c0, zt);
#pragma unroll
      for (int hb = 0; hb < NHM; ++hb) {
        if (hb >= NHB) continue;
        const int hl = tile_unit(hb) + l16;
        const float bias = b1s[hl];
        float w2v[KO];
#pragma unroll
        for (int k = 0; k < KO; ++k) w2v[k] = w2s[k * HB + hl];
#pragma unroll
        for (int rs = 0; rs < 2; ++rs) {
          const f32x4 z = zt[hb][rs];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float av = hidden_sigmoid<PREC>(z[i] + bias);
#pragma unroll
            for (int k = 0; k < KO; ++k) zp[rs][i][k] = fmaf(av, w2v[k], zp[rs][i][k]);
          }
        }
      }
      // sum over the 16 hidden lanes of each row (fixed butterfly)
#pragma unroll
      for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < KO; ++k) zp[rs][i][k] = sum16(zp[rs][i][k]);
      // consecutive chunks alternate between two buffers, so one barrier per
      // chunk separates the writes of a buffer from the reads of its
      // previous contents (two chunks back)
      float *zw = z2w + ((c0 / kRC) & 1) * (kNW * kRC * 4);
      if (l16 == 0) {
#pragma unroll
        for (int rs = 0; rs < 2; ++rs)
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) zw[(wave * kRC + rs * 16 + 4 * lg + i) * 4 + k] = k < KO ? zp[rs][i][k] : 0.0f;
      }
      __syncthreads();
      for (int q = tid; q < kRC * 4; q += kLT) {
        const int rr = q >> 2, k = q & 3;
        // waves in pairs, then pairs of pairs (a fixed tree)
        float v[kNW];
#pragma unroll
        for (int w = 0; w < kNW; ++w) v[w] = zw[(w * kRC + rr) * 4 + k];
#pragma unroll
        for (int st = 1; st < kNW; st *= 2)
#pragma unroll
          for (int w = 0; w < kNW; w += 2 * st) v[w] += v[w + st];
        out(rr, k, v[0]);
      }
    };

    // The same partial output pre-activations with the work split by rows:
    // one wave takes a 16-row set of the piece and runs z1 for every hidden
    // tile of the block (four tiles at a time), sigma and the output-layer
    // sums, reduced over the tile rows' 16 lanes and across tiles in
    // registers -- no exchange between waves and no workgroup barrier, so the
    // two waves of a SIMD drift apart and one's matrix-core work overlaps the
    // other's sigma.  Used when the piece has a row set for every wave.
    // out(rr, k, v) receives row rr's (within the piece) sum for output k.
    auto z2_rowset = [&](int r0, auto &&out) {
      float zp[4][KO];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < KO; ++k) zp[i][k] = 0.0f;
      float xa32[16];
      bf16x8 xa16[2];
      long xa8[2];
      if (PREC == 0) {
#pragma unroll
        for (int st = 0; st < 16; ++st) xa32[st] = reinterpret_cast<const float *>(xr)[(r0 + l16) * XROW + lg + 4 * st];
      } else if (PREC == 1) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          xa16[ks] = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const __bf16 *>(xr) + (r0 + l16) * XROW +
                                                       8 * lg + 32 * ks);
      } else {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          xa8[ks] = *reinterpret_cast<const long *>(reinterpret_cast<const uint8_t *>(xr) + (r0 + l16) * XROW +
                                                    8 * lg + 32 * ks);
      }
      // Tiles go in groups of 4; a group's tile index is clamped to the block
      // (the products of a clamped tile are computed and dropped).  bf16 /
      // e4m3: the W1 operands of the next group are loaded while this group's
      // sigma runs; float32 (16 operands per tile): the group's 64 operands
      // are loaded together ahead of its products.
      bf16x8 wvb[4][2];
      long wve[4][2];
      auto load_group = [&](int t0) {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int t = min(t0 + tt, NT - 1);
#pragma unroll
          for (int ks = 0; ks < 2; ++ks) {
            const int o = (16 * t + l16) * XROW + 8 * lg + 32 * ks;
            if (PREC == 1) wvb[tt][ks] = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const __bf16 *>(w1s) + o);
            if (PREC == 2) wve[tt][ks] = *reinterpret_cast<const long *>(reinterpret_cast<const uint8_t *>(w1s) + o);
          }
        }
      };
      if (PREC != 0) load_group(0);
      for (int t0 = 0; t0 < NT; t0 += 4) {
        float bias[4], w2v[4][KO];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int hl = 16 * min(t0 + tt, NT - 1) + l16;
          bias[tt] = b1s[hl];
#pragma unroll
          for (int k = 0; k < KO; ++k) w2v[tt][k] = w2s[k * HB + hl];
        }
        f32x4 z[4];
        if (PREC == 0) {
          float wv[4][16];
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const float *wb = reinterpret_cast<const float *>(w1s) + (16 * min(t0 + tt, NT - 1) + l16) * XROW + lg;
#pragma unroll
            for (int st = 0; st < 16; ++st) wv[tt][st] = wb[4 * st];
          }
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) z[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            if (16 * g < DK) {
#pragma unroll
              for (int st = 4 * g; st < 4 * g + 4; ++st)
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
                  z[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa32[st], wv[tt][st], z[tt], 0, 0, 0);
            }
          }
        } else {
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            if (PREC == 1) {
              z[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa16[0], wvb[tt][0], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
              z[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa16[1], wvb[tt][1], z[tt], 0, 0, 0);
            } else {
              z[tt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xa8[0], wve[tt][0], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
              z[tt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xa8[1], wve[tt][1], z[tt], 0, 0, 0);
            }
          }
          if (t0 + 4 < NT) load_group(t0 + 4);
          if (PREC == 2) {
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) z[tt] = z[tt] * (isx * isw);
          }
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          if (t0 + tt < NT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float av = hidden_sigmoid<PREC>(z[tt][i] + bias[tt]);
#pragma unroll
              for (int k = 0; k < KO; ++k) zp[i][k] = fmaf(av, w2v[tt][k], zp[i][k]);
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < KO; ++k) zp[i][k] = sum16(zp[i][k]);
      if (l16 == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < KO; ++k) out(r0 + 4 * lg + i, k, zp[i][k]);
      }
    };
    // row sets of the piece for every wave: split the work by rows
    const bool by_rows = RBP / 16 >= kNW;

    const bool split = a.Gj > 1;
    if (split) {
      // the Gj partials of a row meet in the workspace
      for (int pc = 0; pc < NPc; ++pc) {
        stage_piece(pc);
        const int64_t rowbase = (int64_t)gc * a.b + (int64_t)gi * RB + (int64_t)pc * RBP;
        float *zrow = a.z2p + rowbase * 4;   // this piece's rows (uniform base, 32-bit offsets)
        if (by_rows) {
          for (int r0 = 16 * wave; r0 < RBP; r0 += 16 * kNW)
            z2_rowset(r0, [&](int rr, int k, float v) { zrow[rr * 4 + k] = v; });
        } else {
          for (int c0 = 0; c0 < RBP; c0 += kRC)
            z2_chunk(c0, [&](int rr, int k, float v) { zrow[(c0 + rr) * 4 + k] = v; });
        }
      }
      if (!barrier()) { ok = false; break; }
    }

    // ================================================================ phase 2
    // Per piece of the row block (the split case walks the pieces backwards,
    // starting from the one phase 1 left in LDS): output layer, error and
    // delta2 of its rows, then delta1 and the gradient contributions.
    float sq = 0.0f, gb2 = 0.0f;
    f32x4 gacc[NHM][4];
#pragma unroll
    for (int hb = 0; hb < NHM; ++hb)
#pragma unroll
      for (int fb = 0; fb < 4; ++fb) gacc[hb][fb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float gb1[NHM];
#pragma unroll
    for (int hb = 0; hb < NHM; ++hb) gb1[hb] = 0.0f;
    float gw2[NHM][KO];
#pragma unroll
    for (int hb = 0; hb < NHM; ++hb)
#pragma unroll
      for (int k = 0; k < KO; ++k) gw2[hb][k] = 0.0f;
    float d1max = 0.0f;

    for (int t = 0; t < NPc; ++t) {
      const int pc = split ? NPc - 1 - t : t;
      stage_piece(pc);
      const int prow0 = pc * RBP;                                // first row of the piece in the block
      const int prows = max(0, min(RBP, rows_here - prow0));     // real rows of the piece
      if (!split) {
        // Gj == 1: z2 partials are complete inside this workgroup
        if (by_rows) {
          for (int r0 = 16 * wave; r0 < RBP; r0 += 16 * kNW)
            z2_rowset(r0, [&](int rr, int k, float v) { d2s[rr * 4 + k] = v; });
        } else {
          for (int c0 = 0; c0 < RBP; c0 += kRC)
            z2_chunk(c0, [&](int rr, int k, float v) { d2s[(c0 + rr) * 4 + k] = v; });
        }
        __syncthreads();   // d2s entries are read below by other threads
      }
      {
        // entries (row, output) of this piece, kIt per thread at the largest
        // piece; every load (b2, targets, the Gj partials) is issued before
        // the first use
        constexpr int kIt = 512 * 4 / kLT;
        const float *tb = a.T + (rb0 + prow0) * K;   // the piece's targets
        float zv[kIt], tv[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
          const int q = tid + it * kLT, rr = q >> 2, k = q & 3;
          const bool on = q < RBP * 4 && k < K && rr < prows;
          zv[it] = load_if(th + oB2 + k, th, on);
          tv[it] = load_if(tb + (rr * K + k), a.T, on);
        }
        if (split) {
          const float *zb = a.z2p + ((int64_t)(net * a.Gj) * a.b + (int64_t)gi * RB + prow0) * 4;
#pragma unroll 4
          for (int g = 0; g < a.Gj; ++g) {
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
              const int q = tid + it * kLT, rr = q >> 2, k = q & 3;
              zv[it] += load_if(zb + (int64_t)g * a.b * 4 + q, a.z2p, q < RBP * 4 && k < K && rr < prows);
            }
          }
        } else {
#pragma unroll
          for (int it = 0; it < kIt; ++it) {
            const int q = tid + it * kLT, rr = q >> 2, k = q & 3;
            if (q < RBP * 4 && k < K && rr < prows) zv[it] += d2s[q];
          }
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
          const int q = tid + it * kLT, rr = q >> 2, k = q & 3;
          if (q < RBP * 4) {
            float d = 0.0f;
            if (k < K && rr < prows) {
              const float y = sigmoid(zv[it]);
              const float err = y - tv[it];
              sq = fmaf(err, err, sq);
              d = dscale * err * y * (1.0f - y);
            }
            d2s[q] = d;  // each entry is read and rewritten by the same thread
          }
        }
      }
      __syncthreads();
      // gb2 (hidden block 0 only; other blocks hold copies): wave k sums
      // output k over the piece's rows, lane-strided
      if (gj == 0)
        for (int rr = lane; rr < RBP; rr += 64) gb2 += d2s[rr * 4 + wave];

      // recompute a, form delta1, accumulate gW1 (MFMA), gb1, gW2.  delta1
      // feeds the gW1 contraction straight from registers: the chunk's rows
      // are summed in the order the z1 accumulator holds them (lane group lg
      // has rows 4 lg + i and 16 + 4 lg + i of the chunk), and the X operand
      // is read for the same rows.
      // z1 of the next chunk is issued on the matrix cores before this
      // chunk's vector work (sigma', delta1), which does not depend on it
      f32x4 ztn[NHM][2];
      z1_tiles(0, ztn);
      for (int c0 = 0; c0 < RBP; c0 += kRC) {
      f32x4 zt[NHM][2];
#pragma unroll
      for (int hb = 0; hb < NHM; ++hb) {
        zt[hb][0] = ztn[hb][0];
        zt[hb][1] = ztn[hb][1];
      }
      if (c0 + kRC < RBP) z1_tiles(c0 + kRC, ztn);
      // X operands of this chunk's gW1 contraction, shared by the wave's tiles:
      // float32 [rs][i][fb] = X[c0 + 16 rs + 4 lg + i][16 fb + l16]; bf16 /
      // e4m3 [fb] = X[rows c0 + 4 lg .. +3, then c0 + 16 + 4 lg .. +3][16 fb + l16]
      float xg[2][4][4];
      bf16x8 xgb[4];
      long xge[4];
      if (PREC == 0) {
#pragma unroll
        for (int rs = 0; rs < 2; ++rs)
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
              xg[rs][i][fb] = reinterpret_cast<const float *>(xr)[(c0 + 16 * rs + 4 * lg + i) * XROW + 16 * fb + l16];
      } else if (PREC == 1) {
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
          const __bf16 *p = reinterpret_cast<const __bf16 *>(xt) + (16 * fb + l16) * XTS + c0 + 4 * lg;
          typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
          const bf16x4 lo = *reinterpret_cast<const bf16x4 *>(p);
          const bf16x4 hi = *reinterpret_cast<const bf16x4 *>(p + 16);
          xgb[fb] = bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        }
      } else {
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
          const uint8_t *p = reinterpret_cast<const uint8_t *>(xt) + (16 * fb + l16) * XTS + c0 + 4 * lg;
          const uint32_t lo = *reinterpret_cast<const uint32_t *>(p);
          const uint32_t hi = *reinterpret_cast<const uint32_t *>(p + 16);
          xge[fb] = (long)((uint64_t)lo | ((uint64_t)hi << 32));
        }
      }
#pragma unroll
      for (int hb = 0; hb < NHM; ++hb) {
        if (hb < NHB) {
          const int hl = tile_unit(hb) + l16;
          const float bias = b1s[hl];
          float w2v[KO];
#pragma unroll
          for (int k = 0; k < KO; ++k) w2v[k] = w2s[k * HB + hl];
          float d1v[2][4];
#pragma unroll
          for (int rs = 0; rs < 2; ++rs) {
            const f32x4 z = zt[hb][rs];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int rr = rs * 16 + 4 * lg + i;          // row within the chunk
              float slope;
              const float av = hidden_sigmoid_slope<PREC>(z[i] + bias, slope);
              const float4 dv = *reinterpret_cast<const float4 *>(d2s + (c0 + rr) * 4);
              const float dd[4] = {dv.x, dv.y, dv.z, dv.w};
              float bp = 0.0f;
#pragma unroll
              for (int k = 0; k < KO; ++k) {
                bp = fmaf(dd[k], w2v[k], bp);
                gw2[hb][k] = fmaf(dd[k], av, gw2[hb][k]);
              }
              const float d1 = bp * slope;
              gb1[hb] += d1;
              d1v[rs][i] = d1;
              if (PREC == 2) d1max = fmaxf(d1max, fabsf(d1));
              // float32: gW1[tile][feature blocks] += delta1^T X, one k-step
              // per row as soon as its delta1 is formed, so the products of
              // one row run on the matrix cores under the next row's vector
              // work (the feature blocks are independent accumulators; blocks
              // past D multiply the zero LDS padding and are never stored)
              if (PREC == 0) {
#pragma unroll
                for (int fb = 0; fb < 4; ++fb)
                  gacc[hb][fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(d1, xg[rs][i][fb], gacc[hb][fb], 0, 0, 0);
              }
            }
          }
          // bf16 / e4m3: gW1[tile][feature blocks] += delta1^T X over the chunk's rows
          if (PREC == 1) {
            bf16x8 av;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              av[j] = (__bf16)d1v[0][j];
              av[4 + j] = (__bf16)d1v[1][j];
            }
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
              gacc[hb][fb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, xgb[fb], gacc[hb][fb], 0, 0, 0);
          } else if (PREC == 2) {
            const long av =
                (long)((uint64_t)pack_e4m3x4(d1v[0][0] * sd, d1v[0][1] * sd, d1v[0][2] * sd, d1v[0][3] * sd) |
                       ((uint64_t)pack_e4m3x4(d1v[1][0] * sd, d1v[1][1] * sd, d1v[1][2] * sd, d1v[1][3] * sd) << 32));
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
              gacc[hb][fb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, xge[fb], gacc[hb][fb], 0, 0, 0);
          }
        }
      }
    }
    }  // pieces

    // loss and gb2 partials of this net's row block (hidden block 0 only)
    if (gj == 0) {
      for (int off = 32; off >= 1; off >>= 1) gb2 += __shfl_xor(gb2, off, kWave);
      sq = wg_reduce_sum(sq, 0);
      if (tid == 0) a.lossp[(int64_t)gi * a.M + net] = sq;
      if (lane == 0 && wave < K) a.gp[(int64_t)gi * PT + (int64_t)net * P + oB2 + wave] = gb2;
    }

    // write this workgroup's partial gradients
    {
      float *gpi = a.gp + (int64_t)gi * PT + (int64_t)net * P;
      const float gscale = PREC == 2 ? isd * isx : 1.0f;
      // lane coordinates made opaque to the compiler here, so the store
      // addresses below are formed per step next to their stores instead of
      // being hoisted out of the step loop (where they would sit in
      // registers, or in scratch, for the whole run)
      int lg_o = lg, l16_o = l16;
      asm volatile("" : "+v"(lg_o), "+v"(l16_o));
#pragma unroll
      for (int hb = 0; hb < NHM; ++hb) {
        if (hb < NHB) {
#pragma unroll
          for (int fb = 0; fb < 4; ++fb) {
            if (fb < NFB) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int h = gj * HB + (hb * kNW + wave) * 16 + 4 * lg_o + i, d = fb * 16 + l16_o;
                if (h < H && d < D) gpi[h * D + d] = gacc[hb][fb][i] * gscale;
              }
            }
          }
          float v = gb1[hb];
          v += __shfl_xor(v, 16, kWave);
          v += __shfl_xor(v, 32, kWave);
          float w[KO];
#pragma unroll
          for (int k = 0; k < KO; ++k) {
            float t = gw2[hb][k];
            t += __shfl_xor(t, 16, kWave);
            t += __shfl_xor(t, 32, kWave);
            w[k] = t;
          }
          const int h = gj * HB + (hb * kNW + wave) * 16 + l16_o;
          if (lg_o == 0 && h < H) {
            gpi[oB1 + h] = v;
#pragma unroll
            for (int k = 0; k < KO; ++k)
              if (k < K) gpi[oW2 + (int64_t)k * H + h] = w[k];
          }
        }
      }
      if (PREC == 2) {
        d1max = wg_reduce_max(d1max, 8);
        if (tid == 0) a.amax[2 * G + (step & 1) * G + bid] = d1max;
      }
    }
    if (!barrier()) { ok = false; break; }

    // ================================================================ phase 3
    // Sum the Gi partials of this workgroup's slice of the parameters (of all
    // nets) in a fixed order and update the master copy.  Lanes run over
    // parameters (coalesced reads of each partial row); with few parameters
    // per workgroup the waves split the partials and meet in LDS.
    {
      const int64_t per = (PT + G - 1) / G;
      const int64_t p0 = (int64_t)bid * per;
      const int np = (int)max((int64_t)0, min(PT, p0 + per) - p0);
      float wmax = 0.0f;
      auto update = [&](int64_t p, float w, float c, float gsum) {
        const float lr = a.M == 1 ? a.lr[0] : a.lr[(int)(p / P)];
        gd_update(w, c, lr, gsum, a.comp != nullptr);
        a.theta[p] = w;
        if (PREC == 1 && a.w1h != nullptr) reinterpret_cast<__bf16 *>(a.w1h)[p] = (__bf16)w;
        if (a.comp) a.comp[p] = c;
        if (p < oB1) wmax = fmaxf(wmax, fabsf(w));
      };
      // sum of partials g in [g0, g1) of parameter p, in increasing g; the
      // loads of a batch are all issued before the first add.  g0 and g1 are
      // uniform over the wave, so the batches need no lane masks; each load
      // is a uniform partial-row base plus the lane's 32-bit byte offset
      // (Gi PT < 2^30 floats).
      auto psum = [&](int64_t p, int g0, int g1) {
        g0 = __builtin_amdgcn_readfirstlane(g0);
        g1 = __builtin_amdgcn_readfirstlane(g1);
        uint32_t pq = (uint32_t)p * 4u;
        asm volatile("" : "+v"(pq));   // formed per step (see the gradient stores)
        const char *gpb = reinterpret_cast<const char *>(a.gp);
        const uint64_t rowb = (uint64_t)PT * 4u;
        float sum = 0.0f;
        int gb = g0;
        for (; gb + kRedU <= g1; gb += kRedU) {
          const char *base = gpb + (uint64_t)gb * rowb;
          float v[kRedU];
#pragma unroll
          for (int u = 0; u < kRedU; ++u) v[u] = *reinterpret_cast<const float *>(base + u * rowb + pq);
#pragma unroll
          for (int u = 0; u < kRedU; ++u) sum += v[u];
        }
        if (gb < g1) {
          // the last, partial batch: a partial past g1 (uniform test) reads
          // partial g0 instead and adds zero, so every load is issued at once
          const char *base = gpb + (uint64_t)gb * rowb, *safe = gpb + (uint64_t)g0 * rowb;
          float v[kRedU];
#pragma unroll
          for (int u = 0; u < kRedU; ++u)
            v[u] = *reinterpret_cast<const float *>((gb + u < g1 ? base + u * rowb : safe) + pq);
#pragma unroll
          for (int u = 0; u < kRedU; ++u) sum += gb + u < g1 ? v[u] : 0.0f;
        }
        return sum;
      };
      if (np <= 64 && a.Gi >= kNW) {
        // few parameters, many partials: the waves split the partials and
        // meet in LDS (fixed tree)
        const int g0 = (a.Gi * wave) / kNW, g1 = (a.Gi * (wave + 1)) / kNW;
        float w = 0.0f, c = 0.0f, sum = 0.0f;
        if (lane < np) {
          if (wave == 0) {
            w = a.theta[p0 + lane];
            c = a.comp ? a.comp[p0 + lane] : 0.0f;
          }
          sum = psum(p0 + lane, g0, g1);
        }
        z2w[wave * 64 + lane] = sum;
        __syncthreads();
        if (wave == 0 && lane < np) {
          float v[kNW];
#pragma unroll
          for (int w8 = 0; w8 < kNW; ++w8) v[w8] = z2w[w8 * 64 + lane];
#pragma unroll
          for (int st = 1; st < kNW; st *= 2)
#pragma unroll
            for (int w8 = 0; w8 < kNW; w8 += 2 * st) v[w8] += v[w8 + st];
          update(p0 + lane, w, c, v[0]);
        }
      } else if (a.Gi <= 4) {
        // many parameters, at most 4 partials each (nets sharing X): kUpdU
        // parameters per thread per batch, all their loads issued together
        for (int q0 = 0; q0 < np; q0 += kUpdU * kLT) {
          float w[kUpdU], c[kUpdU], v[kUpdU][4];
#pragma unroll
          for (int u = 0; u < kUpdU; ++u) {
            const int q = q0 + u * kLT + tid;
            const bool on = q < np;
            const int64_t pp = p0 + (on ? q : 0);
            w[u] = a.theta[pp];
            c[u] = a.comp ? a.comp[pp] : 0.0f;
#pragma unroll
            for (int g = 0; g < 4; ++g) v[u][g] = load_if(a.gp + (int64_t)g * PT + pp, a.gp, g < a.Gi);
          }
#pragma unroll
          for (int u = 0; u < kUpdU; ++u) {
            const int q = q0 + u * kLT + tid;
            if (q < np) {
              float sum = v[u][0];
#pragma unroll
              for (int g = 1; g < 4; ++g)
                if (g < a.Gi) sum += v[u][g];
              update(p0 + q, w[u], c[u], sum);
            }
          }
        }
      } else {
        // one parameter per thread, all of its partials in flight at once
        for (int q = tid; q < np; q += kLT) {
          const float w = a.theta[p0 + q], c = a.comp ? a.comp[p0 + q] : 0.0f;
          update(p0 + q, w, c, psum(p0 + q, 0, a.Gi));
        }
      }
      if (PREC == 2) {
        wmax = wg_reduce_max(wmax, 16);
        if (tid == 0) a.amax[((step + 1) & 1) * G + bid] = wmax;
      }
      if (bid < a.M && wave == 0) {
        // workgroup n keeps net n's loss: lanes take every 64th row block,
        // then a fixed butterfly
        float sl = 0.0f;
        for (int g = lane; g < a.Gi; g += kWave) sl += a.lossp[(int64_t)g * a.M + bid];
        sl = wave_sum(sl);
        if (lane == 0) {
          const float lstep = sl / ((float)m * (float)K);
          const float accum = (sidx == 0 ? 0.0f : a.acc[bid]) + lstep;
          a.acc[bid] = accum;
          if (sidx == a.steps_per_epoch - 1 && a.loss_hist)
            a.loss_hist[(int64_t)bid * a.epochs + e] = accum / (float)a.steps_per_epoch;
        }
      }
    }
    if (!barrier()) { ok = false; break; }
  }
  // a wait gave up: every workgroup has left the step loop; the losses of
  // the epoch that failed and of every later epoch are NaN (the parameters
  // may hold a partial update; the host reads the give-up word)
  if (!ok && bid < a.M && tid == 0 && a.loss_hist) {
    const int e0 = min(step, total_steps - 1) / a.steps_per_epoch;
    for (int e = max(e0, 0); e < a.epochs; ++e) a.loss_hist[(int64_t)bid * a.epochs + e] = __builtin_nanf("");
  }
}

__global__ void k_zero_u32(unsigned *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// Grid-barrier probe: the workgroups of a co-resident grid pass `rounds`
// grid barriers of the trainer's kind and do nothing else, so a launch's
// time over its rounds is the latency one barrier adds to a step when every
// workgroup arrives together (the trainer pays three per step, plus the
// wait for its slowest workgroup).
__global__ __launch_bounds__(kProbeLT) void k_barrier_probe(unsigned *bar, int rounds, uint64_t wait_limit) {
  __shared__ int ok_s;
  GridSync gs;
  if (threadIdx.x == 0) ok_s = gs.init(bar, gridDim.x, wait_limit) ? 1 : 0;
  __syncthreads();
  for (int r = 0; r < rounds && ok_s; ++r) {
    __syncthreads();
    if (threadIdx.x == 0 && !gs.arrive_and_wait()) ok_s = 0;
    __syncthreads();
  }
}

// Finite check (MLP_F_CHECK_FINITE): a nonzero word `flag` if any of
// a[0..na) or b[0..nb) is NaN or infinite.  Every writer stores the same
// value, so the race between writers is harmless.
__global__ void k_check_finite(const float *a, int64_t na, const float *b, int64_t nb, unsigned *flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
    const float v = i < na ? a[i] : b[i - na];
    bad |= !__builtin_isfinite(v);
  }
  if (bad) *flag = 1u;
}

// Contraction probe: C[m][n] = sum_k A[m][k] B[n][k] on the matrix-core
// instruction the trainer uses for the operand format PREC, with the same
// operand layout and the same chained float32 accumulation over k (steps of
// 4 for float32, 32 for bf16 / e4m3).  Operands arrive as float32 values and
// are converted to the format (exact when the caller passes representable
// values), so the result differs from the exact sum only by the matrix
// core's own summation.  One wave per 16 x 16 tile of C.
template <int PREC>
__global__ __launch_bounds__(64) void k_mfma_probe(const float *A, const float *B, float *C, int M, int N, int Kd) {
  const int lane = threadIdx.x, l16 = lane & 15, lg = lane >> 4;
  const int tiles_n = N / 16;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const float *a = A + (int64_t)(tm * 16 + l16) * Kd;
  const float *b = B + (int64_t)(tn * 16 + l16) * Kd;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (PREC == 0) {
    for (int k0 = 0; k0 < Kd; k0 += 4) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k0 + lg], b[k0 + lg], acc, 0, 0, 0);
  } else if (PREC == 1) {
    for (int k0 = 0; k0 < Kd; k0 += 32) {
      bf16x8 av, bv;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        av[j] = (__bf16)a[k0 + 8 * lg + j];
        bv[j] = (__bf16)b[k0 + 8 * lg + j];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < Kd; k0 += 32) {
      const float *pa = a + k0 + 8 * lg, *pb = b + k0 + 8 * lg;
      const long av = (long)pack_e4m3x4(pa[0], pa[1], pa[2], pa[3]) | ((long)pack_e4m3x4(pa[4], pa[5], pa[6], pa[7]) << 32);
      const long bv = (long)pack_e4m3x4(pb[0], pb[1], pb[2], pb[3]) | ((long)pack_e4m3x4(pb[4], pb[5], pb[6], pb[7]) << 32);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) C[(int64_t)(tm * 16 + 4 * lg + i) * N + tn * 16 + l16] = acc[i];
}

}  // namespace mlpk

namespace mlph {

namespace {

constexpr int kMaxRowBlocks = 256, kMaxHiddenBlocks = 16;
constexpr size_t kLdsLimit = 160 * 1024;
int g_grid_rows = 0, g_grid_hidden = 0, g_waves = 0;  // launch hint (0: automatic)
constexpr int64_t kDefaultWaitUs = 5000000;  // a grid-barrier wait gives up after 5 s
int64_t g_wait_us = kDefaultWaitUs;

// Microseconds -> ticks of the device's constant-rate wall clock.
uint64_t wait_ticks(std::string *err, bool *ok) {
  int dev = 0, khz = 0;
  *ok = hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0;
  if (!*ok) {
    *err = "could not read the device wall-clock rate";
    return 0;
  }
  return (uint64_t)g_wait_us * (uint64_t)khz / 1000u;
}

struct Plan {
  int Gi, Gj, Hp, RBP;
  int nw;   // waves per workgroup (4 or 8)
  size_t lds;
};

template <int PREC>
size_t lds_bytes(int HB, int RB) {
  return (size_t)mlpk::LLayout<PREC>(HB, RB).total();
}

size_t lds_for(int prec, int HB, int RB) {
  if (prec == 0) return lds_bytes<0>(HB, RB);
  if (prec == 1) return lds_bytes<1>(HB, RB);
  return lds_bytes<2>(HB, RB);
}

// Rows staged in LDS at a time: the largest multiple of 32 that divides the
// row block, is at most 512 and fits the LDS budget with the hidden block
// (0: none).
int piece_rows(int prec, int HB, int RB, size_t limit) {
  for (int r = std::min(RB, 512) / 32 * 32; r >= 32; r -= 32)
    if (RB % r == 0 && lds_for(prec, HB, r) <= limit) return r;
  return 0;
}

int64_t batch_of(const mlp_config &c) { return (c.batch <= 0 || c.batch >= c.n_rows) ? c.n_rows : c.batch; }

int min_hidden_blocks(int H) {
  int Gj = 1;   // hidden blocks: at most 256 units each (4 waves x 64)
  while ((H + 64 * Gj - 1) / (64 * Gj) * 64 > 256) Gj *= 2;
  return Gj;
}

// Workspace layout (bytes, 256-aligned pieces).  The barrier counters and
// status words come first, so the status of the last launch sits at a fixed
// place (mlp_workspace_status reads it).
struct WsLayout {
  size_t bar, z2p, gp, lossp, amax, acc, w1h, total;
};

WsLayout ws_layout(const mlp_config &c, int M, int Gi, int Gj) {
  const int64_t b = batch_of(c);
  const int64_t P = (int64_t)c.n_in * c.n_hidden + c.n_hidden + (int64_t)c.n_hidden * c.n_out + c.n_out;
  const int64_t bp = (b + 31) / 32 * 32 * 2;   // rows padded for any Gi that divides the block
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  WsLayout w{};
  size_t o = 0;
  static_assert(sizeof(unsigned) * mlpk::kBarWords <= kStatusBytes, "status block");
  w.bar = o; o += kStatusBytes;
  w.z2p = o; o += up(sizeof(float) * (size_t)M * Gj * bp * 4);
  w.gp = o; o += up(sizeof(float) * (size_t)Gi * M * P);
  w.lossp = o; o += up(sizeof(float) * (size_t)Gi * M);
  w.amax = o; o += up(sizeof(float) * (size_t)5 * Gi * M * Gj);
  w.acc = o; o += up(sizeof(float) * (size_t)(M + 4));
  // bf16 operands, one net: the bf16 copy of the parameters the update writes
  w.w1h = 0;
  if (c.prec == MLP_BF16 && M == 1) { w.w1h = o; o += up(sizeof(unsigned short) * (size_t)P); }
  w.total = o;
  return w;
}

// Largest row-block count a plan for M nets may use (one workgroup per CU on
// devices of up to 256 CUs; M > 1 never splits the hidden layer beyond the
// minimum).
int max_row_blocks(int M, int Gj) { return M == 1 ? kMaxRowBlocks : std::max(1, kMaxRowBlocks / (M * Gj)); }

}  // namespace

// Grid shape.  One net: Gj hidden blocks of <= 256 units (a multiple of 64)
// and Gi row blocks of >= 64 rows (>= 32 when the minibatch is smaller),
// Gi*Gj workgroups filling the CUs, with a launch-hint override for the
// autotuner.  (For 4096-row minibatches of a 256-unit layer, 64 row blocks
// x 4 hidden blocks run 5 % faster than 128 x 2: a step there is latency,
// and the longer row blocks halve the partial gradients summed per update.)  M > 1 nets sharing X: each net
// takes the minimum number of hidden blocks, and row blocks are added while
// Gi*M*Gj workgroups still fit one per CU.  Rows of a block are staged in
// LDS in pieces (all of them at once when they fit).
static bool plan_for(const mlp_config &c, int M, int n_cu, Plan *pl, std::string *why) {
  const int64_t b = batch_of(c);
  const int H = c.n_hidden;
  int Gj = min_hidden_blocks(H);
  int Gi = 1;   // row blocks: at least 64 rows each for one net (32 for nets sharing X)
  const int64_t min_rows = (M == 1 && b >= 64) ? 64 : 32;
  while (Gi * 2 * M * Gj <= n_cu && b % (Gi * 2 * min_rows) == 0 && Gi * 2 <= max_row_blocks(M, Gj)) Gi *= 2;
  if (M == 1) {
    // fill the remaining CUs by splitting the hidden layer further
    while (Gi * Gj * 2 <= n_cu && (H + 64 * Gj * 2 - 1) / (64 * Gj * 2) * 64 >= 64 && H > 64 * Gj)
      Gj *= 2;
    if (g_grid_rows > 0 && g_grid_hidden > 0) {
      Gi = g_grid_rows;
      Gj = g_grid_hidden;
    }
  }
  const int Hp = (H + 64 * Gj - 1) / (64 * Gj) * 64 * Gj;
  if (Hp / Gj > 256) { *why = "hidden block above 256 units"; return false; }
  if (Gi > max_row_blocks(M, Gj) || Gj > kMaxHiddenBlocks) { *why = "grid above the workspace plan"; return false; }
  if (b % Gi != 0 || (b / Gi) % 32 != 0) { *why = "rows per block must be a multiple of 32"; return false; }
  // one workgroup per CU: 8 waves (two per SIMD) when the hidden block has
  // a tile for each, else 4
  const int G = Gi * M * Gj;
  if (G > n_cu) { *why = "grid above one workgroup per CU"; return false; }
  pl->Gi = Gi;
  pl->Gj = Gj;
  pl->Hp = Hp;
  pl->nw = g_waves ? g_waves : (Hp / Gj >= 128 ? 8 : 4);
  pl->RBP = piece_rows(c.prec, Hp / Gj, (int)(b / Gi), kLdsLimit);
  if (pl->RBP == 0) { *why = "no row piece of the block fits the LDS"; return false; }
  pl->lds = lds_for(c.prec, Hp / Gj, pl->RBP);
  return true;
}

void set_large_grid_hint(int row_blocks, int hidden_blocks, int waves) {
  g_grid_rows = row_blocks;
  g_grid_hidden = hidden_blocks;
  g_waves = waves;
}

void set_wait_limit_us(int64_t us) { g_wait_us = us < 0 ? kDefaultWaitUs : us; }

static int tiles_per_wave(const Plan &pl);

mlp_status large_plan(const mlp_config &c, int n_nets, int n_cu, int shape[5], std::string *err) {
  if (c.n_in > mlpk::kMaxD || c.n_out > mlpk::kMaxK) {
    *err = "large-N training covers n_in <= 64 and n_out <= 4";
    return MLP_ERR_UNSUPPORTED;
  }
  if (batch_of(c) % 32 != 0) {
    *err = "large-N training needs a minibatch that is a multiple of 32 rows";
    return MLP_ERR_UNSUPPORTED;
  }
  Plan pl;
  std::string why;
  if (!plan_for(c, n_nets, n_cu, &pl, &why)) {
    *err = "no grid for this shape: " + why;
    return MLP_ERR_UNSUPPORTED;
  }
  shape[0] = pl.Gi;
  shape[1] = pl.Gj;
  shape[2] = pl.nw;
  shape[3] = pl.RBP;
  shape[4] = tiles_per_wave(pl);
  return MLP_OK;
}

// The kernel instance: operand type, output count (3 or 4), waves, tiles
// per wave.
template <int NW, int NHM>
static const void *kernel_nw(int prec, bool k3) {
  using namespace mlpk;
  if (prec == MLP_FP32)
    return k3 ? (const void *)k_large_train<0, 3, NW, NHM> : (const void *)k_large_train<0, 4, NW, NHM>;
  if (prec == MLP_BF16)
    return k3 ? (const void *)k_large_train<1, 3, NW, NHM> : (const void *)k_large_train<1, 4, NW, NHM>;
  return k3 ? (const void *)k_large_train<2, 3, NW, NHM> : (const void *)k_large_train<2, 4, NW, NHM>;
}
// tiles per wave of a plan: one when the hidden block has at most one
// 16-unit tile per wave (4 waves), else 16 / waves
static int tiles_per_wave(const Plan &pl) {
  const int nt = pl.Hp / pl.Gj / 16;
  return (pl.nw == 4 && nt <= 4) ? 1 : 16 / pl.nw;
}
static const void *kernel_for(int prec, bool k3, const Plan &pl) {
  if (pl.nw == 8) return kernel_nw<8, 2>(prec, k3);
  return tiles_per_wave(pl) == 1 ? kernel_nw<4, 1>(prec, k3) : kernel_nw<4, 4>(prec, k3);
}

mlp_status large_workspace_bytes(const mlp_config &c, int n_nets, size_t *bytes) {
  if (c.n_in > mlpk::kMaxD || c.n_out > mlpk::kMaxK) return MLP_ERR_UNSUPPORTED;
  if (n_nets < 1 || n_nets > mlpk::kMaxNets) return MLP_ERR_UNSUPPORTED;
  const int64_t b = batch_of(c);
  if (b % 32 != 0) return MLP_ERR_UNSUPPORTED;
  // Size for the largest grid any plan may use.
  size_t best = 0;
  if (n_nets == 1) {
    for (int gj = 1; gj <= kMaxHiddenBlocks; gj *= 2)
      for (int gi = 1; gi <= kMaxRowBlocks; gi *= 2) best = std::max(best, ws_layout(c, 1, gi, gj).total);
  } else {
    const int gj = min_hidden_blocks(c.n_hidden);
    for (int gi = 1; gi <= max_row_blocks(n_nets, gj); gi *= 2)
      best = std::max(best, ws_layout(c, n_nets, gi, gj).total);
  }
  *bytes = best;
  return MLP_OK;
}

mlp_status large_train(const mlp_config &c, int n_nets, const float *lrs, const mlp_params &theta,
                       float *comp, void *ws, size_t ws_bytes, int n_cu, const float *X, const float *T,
                       int epochs, float *loss_hist, hipStream_t s, std::string *err) {
  if (c.n_in > mlpk::kMaxD || c.n_out > mlpk::kMaxK) {
    *err = "large-N trainer supports n_in <= 64 and n_out <= 4";
    return MLP_ERR_UNSUPPORTED;
  }
  if (n_nets < 1 || n_nets > mlpk::kMaxNets) {
    *err = "between 1 and " + std::to_string(mlpk::kMaxNets) + " nets may share X";
    return MLP_ERR_UNSUPPORTED;
  }
  if (n_nets > 1 && c.prec == MLP_FP8_E4M3) {
    *err = "nets sharing X train in float32 or bf16 operands (e4m3 scales are per net)";
    return MLP_ERR_UNSUPPORTED;
  }
  const int64_t D = c.n_in, H = c.n_hidden, K = c.n_out;
  if (theta.b1 != theta.W1 + D * H || theta.W2 != theta.b1 + H || theta.b2 != theta.W2 + H * K) {
    *err = "large-N training needs W1, b1, W2, b2 contiguous in packed order";
    return MLP_ERR_UNSUPPORTED;
  }
  const int64_t b = batch_of(c);
  if (b % 32 != 0) {
    *err = "large-N training needs a minibatch that is a multiple of 32 rows";
    return MLP_ERR_UNSUPPORTED;
  }
  Plan pl;
  std::string why;
  if (!plan_for(c, n_nets, n_cu, &pl, &why)) {
    *err = "no grid for this shape: " + why;
    return MLP_ERR_UNSUPPORTED;
  }
  const WsLayout wl = ws_layout(c, n_nets, pl.Gi, pl.Gj);
  if (!ws || ws_bytes < wl.total) {
    *err = "workspace too small for the large-N trainer";
    return MLP_ERR_WORKSPACE;
  }
  char *w = static_cast<char *>(ws);
  mlpk::LargeArgs a{};
  a.X = X;
  a.T = T;
  a.theta = theta.W1;
  a.comp = comp;
  a.loss_hist = loss_hist;
  a.z2p = reinterpret_cast<float *>(w + wl.z2p);
  a.gp = reinterpret_cast<float *>(w + wl.gp);
  a.lossp = reinterpret_cast<float *>(w + wl.lossp);
  a.amax = reinterpret_cast<float *>(w + wl.amax);
  a.acc = reinterpret_cast<float *>(w + wl.acc);
  a.w1h = wl.w1h ? reinterpret_cast<unsigned short *>(w + wl.w1h) : nullptr;
  a.bar = reinterpret_cast<unsigned *>(w + wl.bar);
  a.N = c.n_rows;
  a.b = b;
  a.D = (int)D;
  a.H = (int)H;
  a.Hp = pl.Hp;
  a.K = (int)K;
  a.Gi = pl.Gi;
  a.Gj = pl.Gj;
  a.M = n_nets;
  a.RBP = pl.RBP;
  a.epochs = epochs;
  a.steps_per_epoch = (int)((c.n_rows + b - 1) / b);
  for (int i = 0; i < n_nets; ++i) a.lr[i] = lrs ? lrs[i] : c.lr;
  bool tick_ok = false;
  a.wait_limit = wait_ticks(err, &tick_ok);
  if (!tick_ok) return MLP_ERR_HIP;

  hipLaunchKernelGGL(mlpk::k_zero_u32, dim3(1), dim3(256), 0, s, a.bar, mlpk::kBarWords);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { *err = hipGetErrorString(e); return MLP_ERR_HIP; }

  const void *kern = kernel_for(c.prec, c.n_out <= 3, pl);
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
  if (e != hipSuccess) { *err = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * pl.nw, pl.lds);
  if (e != hipSuccess) { *err = std::string("occupancy query: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  const int G = pl.Gi * n_nets * pl.Gj;
  if (per_cu * n_cu < G) {
    *err = "grid of " + std::to_string(G) + " workgroups cannot be co-resident (" +
           std::to_string(per_cu) + " per CU)";
    return MLP_ERR_UNSUPPORTED;
  }
  void *args[] = {&a};
  e = hipLaunchCooperativeKernel(kern, dim3(G), dim3(64 * pl.nw), args, (unsigned)pl.lds, s);
  if (e != hipSuccess) { *err = std::string("cooperative launch: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  if (c.flags & MLP_F_CHECK_FINITE) {
    const int64_t P = D * H + H + H * K + K;
    hipLaunchKernelGGL(mlpk::k_check_finite, dim3(256), dim3(256), 0, s, (const float *)theta.W1, P * n_nets,
                       (const float *)loss_hist, loss_hist ? (int64_t)epochs * n_nets : (int64_t)0,
                       a.bar + mlpk::kNonFiniteWord);
    e = hipGetLastError();
    if (e != hipSuccess) { *err = std::string("finite check: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  }
  return MLP_OK;
}

hipError_t launch_check_finite(const float *a, int64_t na, const float *b, int64_t nb, void *status_block,
                               hipStream_t s) {
  hipLaunchKernelGGL(mlpk::k_check_finite, dim3(256), dim3(256), 0, s, a, na, b, nb,
                     static_cast<unsigned *>(status_block) + mlpk::kNonFiniteWord);
  return hipGetLastError();
}

hipError_t launch_clear_status(void *status_block, hipStream_t s) {
  hipLaunchKernelGGL(mlpk::k_zero_u32, dim3(1), dim3(256), 0, s, static_cast<unsigned *>(status_block),
                     mlpk::kBarWords);
  return hipGetLastError();
}

mlp_status read_status(const void *status_block, hipStream_t s, std::string *err) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) { *err = std::string("stream synchronize: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  unsigned w[2] = {0u, 0u};
  e = hipMemcpy(&w[0], static_cast<const unsigned *>(status_block) + mlpk::kGiveUpWord, sizeof(unsigned),
                hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(&w[1], static_cast<const unsigned *>(status_block) + mlpk::kNonFiniteWord, sizeof(unsigned),
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) { *err = std::string("status read: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  if (w[0]) {
    *err = "a grid-barrier wait of the last training launch gave up: its parameters and losses are not valid";
    return MLP_ERR_TIMEOUT;
  }
  if (w[1]) {
    *err = "the finite check found a NaN or infinite parameter or loss after the last training launch";
    return MLP_ERR_NONFINITE;
  }
  return MLP_OK;
}

mlp_status barrier_probe(int n_wg, int rounds, void *ws, hipStream_t s, std::string *err) {
  unsigned *bar = static_cast<unsigned *>(ws);
  hipLaunchKernelGGL(mlpk::k_zero_u32, dim3(1), dim3(256), 0, s, bar, mlpk::kBarWords);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { *err = hipGetErrorString(e); return MLP_ERR_HIP; }
  bool tick_ok = false;
  uint64_t limit = wait_ticks(err, &tick_ok);
  if (!tick_ok) return MLP_ERR_HIP;
  void *args[] = {&bar, &rounds, &limit};
  e = hipLaunchCooperativeKernel((const void *)mlpk::k_barrier_probe, dim3(n_wg), dim3(mlpk::kProbeLT), args, 0,
                                 s);
  if (e != hipSuccess) { *err = std::string("cooperative launch: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  return MLP_OK;
}

size_t barrier_probe_workspace_bytes() { return sizeof(unsigned) * mlpk::kBarWords; }

// ---------------------------------------------------------------- allocation-free entry
// Scratch of mlp_train_shared_static: device memory of fixed size in the
// code object, one copy per GPU the library is loaded on.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in):
// its device address is looked up once per device and kept.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

mlp_status scratch_of_current_device(void **out, std::string *err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { *err = std::string("hipGetDevice: ") + hipGetErrorString(e); return MLP_ERR_HIP; }
  if (dev < 0 || dev >= kMaxDevices) { *err = "device index above the supported 64"; return MLP_ERR_UNSUPPORTED; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return MLP_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MLP_OK;
}
}  // namespace

mlp_status large_train_static(const mlp_config &c, int n_nets, const float *lrs, const mlp_params &theta,
                              float *comp, int n_cu, const float *X, const float *T, int epochs, float *loss_hist,
                              hipStream_t s, std::string *err) {
  Plan pl;
  std::string why;
  if (!plan_for(c, n_nets, n_cu, &pl, &why)) {
    *err = "no grid for this shape: " + why;
    return MLP_ERR_UNSUPPORTED;
  }
  const size_t need = ws_layout(c, n_nets, pl.Gi, pl.Gj).total;
  if (need > kStaticScratchBytes) {
    *err = "this shape needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
           std::to_string(kStaticScratchBytes) + " (use mlp_train_shared with a workspace)";
    return MLP_ERR_WORKSPACE;
  }
  void *ws = nullptr;
  const mlp_status st = scratch_of_current_device(&ws, err);
  if (st != MLP_OK) return st;
  return large_train(c, n_nets, lrs, theta, comp, ws, kStaticScratchBytes, n_cu, X, T, epochs, loss_hist, s, err);
}

hipError_t launch_mfma_probe(int prec, const float *A, const float *B, float *C, int M, int N, int Kd,
                             hipStream_t s) {
  const dim3 grid((unsigned)((M / 16) * (N / 16)));
  if (prec == MLP_FP32) hipLaunchKernelGGL(mlpk::k_mfma_probe<0>, grid, dim3(64), 0, s, A, B, C, M, N, Kd);
  else if (prec == MLP_BF16) hipLaunchKernelGGL(mlpk::k_mfma_probe<1>, grid, dim3(64), 0, s, A, B, C, M, N, Kd);
  else hipLaunchKernelGGL(mlpk::k_mfma_probe<2>, grid, dim3(64), 0, s, A, B, C, M, N, Kd);
  return hipGetLastError();
}

}  // namespace mlph
