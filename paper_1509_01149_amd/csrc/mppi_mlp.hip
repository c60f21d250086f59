// Learned dynamics on BF16 MFMA (gfx950 v_mfma_f32_16x16x32_bf16): a fused training step
// (forward, loss, backward and the weight-gradient products of 64 samples per block, their
// partial sums reduced with the Adam update in a second kernel) and the fused MPPI rollout
// whose network weights stay in registers for the whole horizon.
// Contract: include/mppi.h, "Learned dynamics".
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

#include "../../include/mppi.h"
#include "mppi_runtime.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace mppi {

constexpr int kH = 128, kIn = 16, kOut = 12;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kOut * kH, kNParams = kOffB3 + kOut;
static_assert(kNParams == MPPI_MLP_PARAMS, "parameter layout");
constexpr int kFrags = 8 + 32 + 4;   // A-operand fragments per lane in the rollout: W1, W2, W3

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// tanh in FP32 as sign(x) (1 - 2 / (exp(2|x|) + 1)) with the hardware exp2 and reciprocal:
// absolute error ~1e-7, below the bfloat16 step of every activation it feeds.
__device__ __forceinline__ float tanh_f(float x) {
  const float e = __builtin_amdgcn_exp2f(2.88539008177792681f * fabsf(x));   // exp(2|x|)
  return copysignf(1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f), x);
}
// tanh(x) from t = 2 log2(e) x, as 1 - 2 / (2^t + 1): valid for either sign (2^t -> 0 gives
// -1, 2^t -> inf gives 1) and the same accuracy as tanh_f; the rollout forms t with one FMA
// from the accumulator and the pre-scaled bias.
constexpr float kTanhScale = 2.88539008177792681f;
__device__ __forceinline__ float tanh_from_scaled(float t) {
  return 1.f - 2.f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(t) + 1.f);
}

// Layer-1 k slot (8 q + e) -> input feature (4 q + e, e < 4) or -1 (zero padding): each lane
// of a 16-sample wave owns four consecutive features of its sample.
__host__ __device__ __forceinline__ int feature_of(int k) {
  const int q = k >> 3, e = k & 7;
  return e < 4 ? 4 * q + e : -1;
}
// Hidden-layer k slot (32 s + 8 q + e) -> hidden unit 16 (2 s + e / 4) + 4 q + e % 4: the unit the
// same lane holds in the previous layer's accumulator, so activations never leave registers.
__host__ __device__ __forceinline__ int hidden_of(int k) {
  const int s = k >> 5, q = (k >> 3) & 3, e = k & 7;
  return 16 * (2 * s + (e >> 2)) + 4 * q + (e & 3);
}

// Dataset: z = (x, u) -> Z [n][16] FP32; dx = dt f(x, u) with the analytic model in FP64 -> D [n][12].
static __global__ void dataset_kernel(const double *x, const double *u, long n, double dt,
                                      const QuadrotorSys::Params p, float *Z, float *D) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xl[12], ul[4], xd[12];
  for (int r = 0; r < 12; ++r) xl[r] = x[i * 12 + r];
  for (int r = 0; r < 4; ++r) ul[r] = u[i * 4 + r];
  QuadrotorSys::xdot(p, xl, ul, xd);
  for (int r = 0; r < 12; ++r) Z[i * 16 + r] = (float)xl[r];
  for (int r = 0; r < 4; ++r) Z[i * 16 + 12 + r] = (float)ul[r];
  for (int r = 0; r < 12; ++r) D[i * 12 + r] = (float)(dt * xd[r]);
}

// Column sums and sums of squares (FP64) of Z (16 columns) and D (12): one block per column.
static __global__ __launch_bounds__(256) void moments_kernel(const float *Z, const float *D, long n, double *out) {
  __shared__ double red[4];
  const int c = blockIdx.x;   // 0..27
  double s = 0.0, s2 = 0.0;
  for (long r = threadIdx.x; r < n; r += 256) {
    const double v = c < 16 ? (double)Z[r * 16 + c] : (double)D[r * 12 + (c - 16)];
    s += v;
    s2 += v * v;
  }
  const double S = block_sum(s, red);
  const double S2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    const double mu = S / (double)n;
    double var = S2 / (double)n - mu * mu;
    double sd = var > 0.0 ? sqrt(var) : 0.0;
    if (!(sd > 0.0)) sd = 1.0;
    const int base = c < 16 ? 0 : 32 - 16;
    out[base + c] = mu;
    out[base + c + (c < 16 ? 16 : 12)] = sd;
  }
}

// Standardise host-side inputs for forward / loss kernels: Zf [B][16] FP64 -> bf16.
static __global__ void std_inputs_kernel(const double *x, const double *u, const double *stats, int B, __bf16 *Xh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * 16) return;
  const int r = i >> 4, c = i & 15;
  const double v = c < 12 ? x[r * 12 + c] : u[r * 4 + c - 12];
  Xh[i] = to_bf16((float)((v - stats[c]) / stats[16 + c]));
}

static __global__ void dx_out_kernel(const float *Yc, const float *b3, const double *stats, int B, double *dx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kOut) return;
  const int c = i % kOut;
  dx[i] = ((double)Yc[i] + (double)b3[c]) * stats[44 + c] + stats[32 + c];
}

// Pack the rollout's A-operand fragments: frag[f][lane][8] bf16 for
//   f in [0, 8):   W1 M-tile f       A[i][k] = W1[16 f + i][feature_of(k)]
//   f in [8, 40):  W2 M-tile t, k-step s (f = 8 + 4 t + s): W2[16 t + i][hidden_of(32 s + k)]
//   f in [40, 44): W3 k-step s       A[i][k] = W3[i][hidden_of(32 s + k)] (rows >= 12 zero)
// where lane l holds row i = l % 16 and k = 8 (l / 16) + e.
static __global__ void pack_rollout_kernel(const float *p, __bf16 *frag) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // over kFrags * 64 * 8
  if (idx >= kFrags * 64 * 8) return;
  const int e = idx & 7, l = (idx >> 3) & 63, f = idx >> 9;
  const int i = l & 15, k = 8 * (l >> 4) + e;
  float v = 0.f;
  if (f < 8) {
    const int c = feature_of(k);
    v = c >= 0 ? p[kOffW1 + (16 * f + i) * kIn + c] : 0.f;
  } else if (f < 40) {
    const int t = (f - 8) >> 2, s = (f - 8) & 3;
    v = p[kOffW2 + (16 * t + i) * kH + hidden_of(32 * s + k)];
  } else {
    const int s = f - 40;
    v = i < kOut ? p[kOffW3 + i * kH + hidden_of(32 * s + k)] : 0.f;
  }
  frag[idx] = to_bf16(v);
}

// ---------------------------------------------------------------- fused training step
// One block = 64 samples (16 per wave).  Each wave runs its samples' forward and backward with
// the weights as the MFMA A operand and the samples as the N dimension, so activations and
// their gradients stay in registers in the accumulator layout (lane (q, n) holds rows 4q..4q+3
// of sample n of every 16-row tile).  The weight gradients are sums over samples: each wave
// writes its operands transposed ([row][sample], bfloat16) into LDS, and the block multiplies
// them with the samples as the K dimension, giving its partial gradient; the bias gradients
// are FP64 sums of the FP32 values over the block's samples.  A second kernel sums the blocks'
// partials in block order and applies Adam.
//
// Fragments ([kTrainFrags][64 lanes] bf16x8, A operands; lane l holds row l % 16 and k slots
// 8 (l / 16) .. + 7):
//   [0, 44):  the forward's, as in the rollout (W1 tiles, W2 tiles x k-steps, W3 k-steps)
//   [44, 52): W3^T tile t: A[i][k] = W3[out_of(k)][16 t + i] (out_of: layer 3's accumulator rows
//             as the B operand delivers them; zero for the padding)
//   [52, 84): W2^T tile t, k-step s (52 + 4 t + s): A[i][k] = W2[hidden_of(32 s + k)][16 t + i]
constexpr int kFwdFrags = 44, kTrainFrags = 84;
constexpr int kTrainSamples = 64;
constexpr int kTS = 72;                    // LDS row stride (bf16) of the transposed operands
constexpr int kNBias = 2 * kH + kOut;      // per-block bias partials: b1 [128], b2 [128], b3 [12]
constexpr int kTrRows = kIn + kH + kH + 16 + kH + kH;   // a0, a1, a2, dY (16 rows), dZ2, dZ1
constexpr int kFBS = kTrainSamples + 1;    // LDS row stride (floats) of the FP32 bias operands
constexpr size_t kTrainLds = (size_t)kTrRows * kTS * 2 + (size_t)kNBias * kFBS * 4;
static_assert((size_t)kTrainFrags * 64 * 16 <= kTrainLds, "fragments fit the operands' LDS");

// Layer 3's accumulator row of B-operand k slot k in a one-k-step product (outputs 4 q .. 4 q + 3
// of lane group q in slots 8 q .. 8 q + 3), or -1 for the zero padding.
__host__ __device__ __forceinline__ int out_of(int k) {
  const int o = feature_of(k);
  return o >= 0 && o < kOut ? o : -1;
}

static __global__ void pack_train_kernel(const float *p, __bf16 *frag) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // over kTrainFrags * 64 * 8
  if (idx >= kTrainFrags * 64 * 8) return;
  const int e = idx & 7, l = (idx >> 3) & 63, f = idx >> 9;
  const int i = l & 15, k = 8 * (l >> 4) + e;
  float v = 0.f;
  if (f < 8) {
    const int c = feature_of(k);
    v = c >= 0 ? p[kOffW1 + (16 * f + i) * kIn + c] : 0.f;
  } else if (f < 40) {
    const int t = (f - 8) >> 2, s = (f - 8) & 3;
    v = p[kOffW2 + (16 * t + i) * kH + hidden_of(32 * s + k)];
  } else if (f < 44) {
    const int s = f - 40;
    v = i < kOut ? p[kOffW3 + i * kH + hidden_of(32 * s + k)] : 0.f;
  } else if (f < 52) {
    const int t = f - 44, o = out_of(k);
    v = o >= 0 ? p[kOffW3 + o * kH + 16 * t + i] : 0.f;
  } else {
    const int t = (f - 52) >> 2, s = (f - 52) & 3;
    v = p[kOffW2 + hidden_of(32 * s + k) * kH + 16 * t + i];
  }
  frag[idx] = to_bf16(v);
}

struct TrainArgs {
  const float *Z, *D;      // dataset [n][16], [n][12] FP32, with order: the minibatch's rows
  const int *order;        // [B] dataset rows, or NULL: inputs from Xh / Tn
  const __bf16 *Xh;        // [B][16] standardised inputs (bfloat16) when order is NULL
  const float *Tn;         // [B][12] standardised targets when order is NULL (backward only)
  const double *stats;     // mu_in, sd_in, mu_out, sd_out
  const float *p;          // FP32 parameters (the biases are read from here)
  const bf16x8 *frag;      // [kTrainFrags][64]
  int B;
  int backward;            // 0: forward only (Yc out), 1: forward, loss and gradient partials
  float *Yc;               // [B][12] W3 a2 without the bias (forward only)
  float *P;                // [blocks][kNParams] weight-gradient partials (bias slots unused)
  double *Pb;              // [blocks][kNBias] bias-gradient partials
  double *Pl;              // [blocks] sums of squared errors
};

static __global__ __launch_bounds__(256) void train_step_kernel(const TrainArgs a) {
  extern __shared__ float4 lds4[];
  __shared__ double red[4];
  bf16x8 *sF = reinterpret_cast<bf16x8 *>(lds4);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4, nn = l & 15;
  const int col = 16 * w + nn;                          // the sample's column in the block
  const int smp = blockIdx.x * kTrainSamples + col;     // its index in the minibatch
  const bool valid = smp < a.B;
  // the fragments into LDS: every load of this thread issued before the first store
  static_assert(kTrainFrags * 64 % 256 == 0, "whole rounds of fragment loads");
  {
    constexpr int kRounds = kTrainFrags * 64 / 256;
    bf16x8 fr[kRounds];
#pragma unroll
    for (int j = 0; j < kRounds; ++j) fr[j] = a.frag[threadIdx.x + 256 * j];
#pragma unroll
    for (int j = 0; j < kRounds; ++j) sF[threadIdx.x + 256 * j] = fr[j];
  }
  // inputs: features 4q..4q+3 of this lane's sample in k slots 8q..8q+3; targets 4q..4q+3
  bf16x8 bz;
  float tgt[4] = {0.f, 0.f, 0.f, 0.f};
  const __bf16 zb = to_bf16(0.f);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    bz[r] = zb;
    bz[4 + r] = zb;
  }
  if (valid) {
    if (a.order) {
      const long row = a.order[smp];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 4 * q + r;
        bz[r] = to_bf16((float)(((double)a.Z[row * 16 + c] - a.stats[c]) / a.stats[16 + c]));
        if (q < 3) tgt[r] = (float)(((double)a.D[row * 12 + c] - a.stats[32 + c]) / a.stats[44 + c]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        bz[r] = a.Xh[(long)smp * 16 + 4 * q + r];
        if (q < 3 && a.backward) tgt[r] = a.Tn[(long)smp * 12 + 4 * q + r];
      }
    }
  }
  __syncthreads();
  // forward: H1 = tanh(W1 a0 + b1), H2 = tanh(W2 a1 + b2), Yc = W3 a2
  float h1[32], h2[32];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sF[t * 64 + l], bz, c, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) h1[4 * t + r] = tanh_f(c[r] + a.p[kOffB1 + 16 * t + 4 * q + r]);
  }
  bf16x8 a1op[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) a1op[s][e] = to_bf16(h1[4 * (2 * s + (e >> 2)) + (e & 3)]);
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sF[(8 + 4 * t + s) * 64 + l], a1op[s], c, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) h2[4 * t + r] = tanh_f(c[r] + a.p[kOffB2 + 16 * t + 4 * q + r]);
  }
  bf16x8 a2op[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) a2op[s][e] = to_bf16(h2[4 * (2 * s + (e >> 2)) + (e & 3)]);
  floatx4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 4; ++s) y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sF[(40 + s) * 64 + l], a2op[s], y, 0, 0, 0);
  if (!a.backward) {
    if (valid && q < 3)
#pragma unroll
      for (int r = 0; r < 4; ++r) a.Yc[(long)smp * kOut + 4 * q + r] = y[r];
    return;
  }
  // loss and its gradient dY = 2 (Y - T) / (12 B); zero for the padding samples and rows
  float g[4];
  double sq = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int o = 4 * q + r;
    g[r] = 0.f;
    if (valid && q < 3) {
      const float d = y[r] + a.p[kOffB3 + o] - tgt[r];
      g[r] = 2.f * d / (float)(a.B * kOut);
      sq = fma((double)d, (double)d, sq);
    }
  }
  bf16x8 gop;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    gop[r] = to_bf16(g[r]);
    gop[4 + r] = zb;
  }
  // dZ2 = (W3^T dY) (1 - H2^2), dZ1 = (W2^T dZ2) (1 - H1^2)
  float dz2[32], dz1[32];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sF[(44 + t) * 64 + l], gop, c, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float h = h2[4 * t + r];
      dz2[4 * t + r] = c[r] * (1.f - h * h);
    }
  }
  bf16x8 dz2op[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) dz2op[s][e] = to_bf16(dz2[4 * (2 * s + (e >> 2)) + (e & 3)]);
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sF[(52 + 4 * t + s) * 64 + l], dz2op[s], c, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float h = h1[4 * t + r];
      dz1[4 * t + r] = c[r] * (1.f - h * h);
    }
  }
  __syncthreads();   // every wave is done with the fragments: their LDS now takes the operands
  __bf16 *T0 = reinterpret_cast<__bf16 *>(lds4);          // a0  [16][kTS]
  __bf16 *T1 = T0 + kIn * kTS;                               // a1  [128][kTS]
  __bf16 *T2 = T1 + kH * kTS;                                // a2  [128][kTS]
  __bf16 *TY = T2 + kH * kTS;                                // dY  [16][kTS]
  __bf16 *TZ2 = TY + 16 * kTS;                               // dZ2 [128][kTS]
  __bf16 *TZ1 = TZ2 + kH * kTS;                              // dZ1 [128][kTS]
  float *FB = reinterpret_cast<float *>(TZ1 + kH * kTS);     // [kNBias][kFBS]: dZ1, dZ2, dY (FP32)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    T0[(4 * q + r) * kTS + col] = valid ? bz[r] : zb;
    TY[(4 * q + r) * kTS + col] = gop[r];
  }
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + 4 * q + r;
      T1[row * kTS + col] = valid ? a1op[t >> 1][4 * (t & 1) + r] : zb;
      T2[row * kTS + col] = valid ? a2op[t >> 1][4 * (t & 1) + r] : zb;
      TZ2[row * kTS + col] = dz2op[t >> 1][4 * (t & 1) + r];
      TZ1[row * kTS + col] = to_bf16(dz1[4 * t + r]);
      FB[row * kFBS + col] = dz1[4 * t + r];
      FB[(kH + row) * kFBS + col] = dz2[4 * t + r];
    }
  if (q < 3)
#pragma unroll
    for (int r = 0; r < 4; ++r) FB[(2 * kH + 4 * q + r) * kFBS + col] = g[r];
  const double loss = block_sum(sq, red);      // its barriers also order the LDS writes above
  if (threadIdx.x == 0) a.Pl[blockIdx.x] = loss;
  // bias partials: FP64 sums over the block's samples, in sample order
  for (int r = threadIdx.x; r < kNBias; r += 256) {
    float fv[kTrainSamples];
#pragma unroll
    for (int c = 0; c < kTrainSamples; ++c) fv[c] = FB[r * kFBS + c];
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < kTrainSamples; ++c) acc += (double)fv[c];
    a.Pb[(long)blockIdx.x * kNBias + r] = acc;
  }
  // weight-gradient partials: sum over the block's 64 samples (two k-steps of 32)
  float *P = a.P + (long)blockIdx.x * kNParams;
  const int ar = l & 15, ak = 8 * (l >> 4);
  // dW2 = dZ2 a1^T: this wave's row tiles 2w, 2w+1 against the eight column tiles
#pragma unroll
  for (int ti = 2 * w; ti < 2 * w + 2; ++ti) {
    floatx4 acc[8];
#pragma unroll
    for (int tj = 0; tj < 8; ++tj) acc[tj] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const bf16x8 A = *reinterpret_cast<const bf16x8 *>(TZ2 + (16 * ti + ar) * kTS + 32 * ks + ak);
#pragma unroll
      for (int tj = 0; tj < 8; ++tj) {
        const bf16x8 Bv = *reinterpret_cast<const bf16x8 *>(T1 + (16 * tj + ar) * kTS + 32 * ks + ak);
        acc[tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv, acc[tj], 0, 0, 0);
      }
    }
#pragma unroll
    for (int tj = 0; tj < 8; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[kOffW2 + (16 * ti + 4 * q + r) * kH + 16 * tj + nn] = acc[tj][r];
  }
  // dW3 = dY a2^T (rows 12..15 of the tile are padding) and dW1 = dZ1 a0^T: tiles 2w, 2w+1
#pragma unroll
  for (int tt = 2 * w; tt < 2 * w + 2; ++tt) {
    floatx4 c3 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const bf16x8 A3 = *reinterpret_cast<const bf16x8 *>(TY + ar * kTS + 32 * ks + ak);
      const bf16x8 B3 = *reinterpret_cast<const bf16x8 *>(T2 + (16 * tt + ar) * kTS + 32 * ks + ak);
      c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A3, B3, c3, 0, 0, 0);
      const bf16x8 A1 = *reinterpret_cast<const bf16x8 *>(TZ1 + (16 * tt + ar) * kTS + 32 * ks + ak);
      const bf16x8 B1 = *reinterpret_cast<const bf16x8 *>(T0 + ar * kTS + 32 * ks + ak);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B1, c1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (q < 3) P[kOffW3 + (4 * q + r) * kH + 16 * tt + nn] = c3[r];
      P[kOffW1 + (16 * tt + 4 * q + r) * kIn + nn] = c1[r];
    }
  }
}

// k slot of the B operand that carries hidden unit h in a k-step product over a hidden layer
// (the inverse of hidden_of): h = 16 (2 s + e / 4) + 4 q + e % 4 at k = 32 s + 8 q + e.
__device__ __forceinline__ int kslot_of_hidden(int h) {
  const int a = h >> 4, rem = h & 15;
  return 32 * (a >> 1) + 8 * (rem >> 2) + 4 * (a & 1) + (rem & 3);
}
// Index of A-operand element (row i, k slot k) of fragment f in the packed array.
__device__ __forceinline__ int frag_slot(int f, int i, int k) { return (f * 64 + 16 * (k >> 3) + i) * 8 + (k & 7); }

// The new value of parameter i into every training fragment that holds it (the inverse of
// pack_train_kernel's mapping; padding slots keep their zeros).
__device__ __forceinline__ void scatter_frag(__bf16 *frag, int i, float v) {
  const __bf16 b = to_bf16(v);
  if (i < kOffB1) {                                   // W1 [128][16]
    const int row = i / kIn, c = i % kIn;
    frag[frag_slot(row >> 4, row & 15, 8 * (c >> 2) + (c & 3))] = b;
  } else if (i >= kOffW2 && i < kOffB2) {             // W2 [128][128]
    const int row = (i - kOffW2) / kH, cj = (i - kOffW2) % kH;
    const int k = kslot_of_hidden(cj), kb = kslot_of_hidden(row);
    frag[frag_slot(8 + 4 * (row >> 4) + (k >> 5), row & 15, k & 31)] = b;
    frag[frag_slot(52 + 4 * (cj >> 4) + (kb >> 5), cj & 15, kb & 31)] = b;
  } else if (i >= kOffW3 && i < kOffB3) {             // W3 [12][128]
    const int o = (i - kOffW3) / kH, h = (i - kOffW3) % kH;
    const int k = kslot_of_hidden(h);
    frag[frag_slot(40 + (k >> 5), o, k & 31)] = b;
    frag[frag_slot(44 + (h >> 4), h & 15, 8 * (o >> 2) + (o & 3))] = b;
  }
}

// Gradient = the blocks' partials summed in a fixed order (each of the four lanes of a quad sums
// every fourth block in block order, then the quad adds its four sums as (l0 + l1) + (l2 + l3);
// weights in FP32, biases in FP64 and then rounded once); with update, Adam on the FP32
// parameters with the bias corrections bias_corr[2 step], bias_corr[2 step + 1] and step size
// *lr (device memory, written before each call, so a captured sequence of steps can be
// replayed), and the new weights scattered into the training fragments.  One quad of lanes per
// parameter; the first wave also sums the loss.
static __global__ void train_reduce_kernel(const float *__restrict__ P, const double *__restrict__ Pb,
                                           const double *__restrict__ Pl, int nblk, int B, float *g, float *p,
                                           float *m, float *v, int update, const float *bias_corr, int step,
                                           const float *lr, __bf16 *frag, double *loss_out) {
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gt >> 2, sub = gt & 3;
  if (blockIdx.x == 0 && threadIdx.x < 64 && loss_out) {
    // the loss: lane j sums blocks j, j + 64, ... in order, then a fixed butterfly over the wave
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += Pl[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double o = __shfl_xor(s, off, 64);
      s = (threadIdx.x & off) ? o + s : s + o;
    }
    if (threadIdx.x == 0) *loss_out = s / (double)(B * kOut);
  }
  if (i >= kNParams) return;                          // whole quads leave together (kNParams quads)
  int bias = -1;
  if (i >= kOffB1 && i < kOffB1 + kH) bias = i - kOffB1;
  else if (i >= kOffB2 && i < kOffB2 + kH) bias = kH + (i - kOffB2);
  else if (i >= kOffB3) bias = 2 * kH + (i - kOffB3);
  float gi;
  if (bias >= 0) {
    // FP64: lane sub sums every fourth block in order, the quad adds (l0 + l1) + (l2 + l3)
    double s = 0.0;
    for (int b = sub; b < nblk; b += 4) s += Pb[(long)b * kNBias + bias];
    const double s1 = __shfl_xor(s, 1, 64);
    const double pair = (sub & 1) ? s1 + s : s + s1;
    const double other = __shfl_xor(pair, 2, 64);
    gi = (float)((sub & 2) ? other + pair : pair + other);
  } else {
    float s = 0.f;
    constexpr int kBatch = 16;                      // loads in flight per lane
    for (int b0 = sub; b0 < nblk; b0 += 4 * kBatch) {
      float t[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) t[j] = b0 + 4 * j < nblk ? P[(long)(b0 + 4 * j) * kNParams + i] : 0.f;
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        if (b0 + 4 * j < nblk) s += t[j];
    }
    const float s1 = __shfl_xor(s, 1, 64);            // the partner's sum (l0 <-> l1, l2 <-> l3)
    const float pair = (sub & 1) ? s1 + s : s + s1;   // l0 + l1 (or l2 + l3) on both lanes
    const float other = __shfl_xor(pair, 2, 64);
    gi = (sub & 2) ? other + pair : pair + other;
  }
  if (sub != 0) return;
  g[i] = gi;
  if (!update) return;
  const float c1 = bias_corr[2 * step], c2 = bias_corr[2 * step + 1];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - *lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  p[i] = pi;
  scatter_frag(frag, i, pi);
}

// ---------------------------------------------------------------- fused rollout
// One wave = 16 samples; lane (q = l / 16, n = l % 16) holds state words 4q..4q+3 of sample n
// (q = 0, 1, 2) or its control (q = 3) -- exactly the slots of the layer-1 operand and of the
// layer-3 accumulator, so the whole step stays in registers.  Weights are loaded once into
// registers (44 bf16x8 fragments per lane).
struct MlpRollArgs {
  const bf16x8 *frag;      // [kFrags][64]
  const float *params;     // FP32 (biases)
  const double *stats;     // mu_in, sd_in, mu_out, sd_out
};

static __global__ __launch_bounds__(256) void mlp_rollout_kernel(const IterArgs a, const QuadrotorSys::Params p,
                                                                 const MlpRollArgs m) {
  extern __shared__ float4 lds4[];
  __shared__ double red[4];
  float *sU = reinterpret_cast<float *>(lds4);    // [T*4]
  float *sRU = sU + a.T * 4;                       // [T*4]
  float *sC = sRU + a.T * 4;                       // [T]
  float *sObs = sU + ((8 * a.T + ((a.T + 3) & ~3) + 3) & ~3);
  const uint64_t it = *a.iter;
  for (int i = threadIdx.x; i < a.T; i += kBlock) {
    float u[4], c = 0.f;
    for (int j = 0; j < 4; ++j) u[j] = a.U32[i * 4 + j];
    for (int r = 0; r < 4; ++r) {
      float s = 0.f;
      for (int j = 0; j < 4; ++j) s += a.R[r * 4 + j] * u[j];
      sU[i * 4 + r] = u[r];
      sRU[i * 4 + r] = s;
      c += u[r] * s;
    }
    sC[i] = 0.5f * c;
  }
  QuadrotorSys::stage(p, sObs, nullptr, nullptr, nullptr);
  __syncthreads();

  const int l = threadIdx.x & 63, q = l >> 4, nn = l & 15;
  const int k = blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + nn;
  bf16x8 W[kFrags];
#pragma unroll
  for (int f = 0; f < kFrags; ++f) W[f] = m.frag[f * 64 + l];
  float b1[32], b2[32];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      b1[4 * t + r] = kTanhScale * m.params[kOffB1 + 16 * t + 4 * q + r];   // pre-scaled biases
      b2[4 * t + r] = kTanhScale * m.params[kOffB2 + 16 * t + 4 * q + r];
    }
  float mu_in[4], isd_in[4], b3[4], sd_out[4], mu_out[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mu_in[r] = (float)m.stats[4 * q + r];
    isd_in[r] = (float)(1.0 / m.stats[16 + 4 * q + r]);
    const int o = 4 * q + r;
    b3[r] = o < kOut ? m.params[kOffB3 + o] : 0.f;
    sd_out[r] = o < kOut ? (float)m.stats[44 + o] : 0.f;
    mu_out[r] = o < kOut ? (float)m.stats[32 + o] : 0.f;
  }
  // own four words: state (q < 3) from x0, control slot (q = 3) filled per step
  float v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = q < 3 ? (float)a.x0[4 * q + r] : 0.f;
  const __bf16 z = to_bf16(0.f);
  double S = 0.0;
  float mine[4];
  for (int i = 0; i < a.T; ++i) {
    // the four lanes of a sample take turns generating its noise: lane q draws the group of
    // step i + q once every four steps; the control lane (q = 3) fetches each step's four.
    if ((i & 3) == 0) normals4((uint32_t)(i + q), (uint32_t)k, it, a.key0, a.key1, mine);
    float e[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) e[c] = __shfl(mine[c], 16 * (i & 3) + nn, 64);
    float du[4] = {0.f, 0.f, 0.f, 0.f};
    if (q == 3) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float t = 0.f;
#pragma unroll
        for (int c = 0; c <= j; ++c) t += a.Ls[j * 4 + c] * e[c];
        du[j] = t;
        v[j] = sU[i * 4 + j] + t;
      }
    }
    // layer 1: H1^T = tanh(W1 zn^T + b1)
    bf16x8 bz;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bz[r] = to_bf16((v[r] - mu_in[r]) * isd_in[r]);
      bz[4 + r] = z;
    }
    float h1[32];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      floatx4 c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[t], bz, c, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[4 * t + r] = tanh_from_scaled(fmaf(c[r], kTanhScale, b1[4 * t + r]));
    }
    bf16x8 b2op[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) b2op[s][e] = to_bf16(h1[4 * (2 * s + (e >> 2)) + (e & 3)]);
    // layer 2
    float h2[32];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[8 + 4 * t + s], b2op[s], c, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[4 * t + r] = tanh_from_scaled(fmaf(c[r], kTanhScale, b2[4 * t + r]));
    }
    bf16x8 b3op[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) b3op[s][e] = to_bf16(h2[4 * (2 * s + (e >> 2)) + (e & 3)]);
    // layer 3: outputs 4q..4q+3 of sample n land in this lane
    floatx4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[40 + s], b3op[s], y, 0, 0, 0);
    if (q < 3) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] += (y[r] + b3[r]) * sd_out[r] + mu_out[r];
    }
    // cost of x_{i+1}: position from lane q = 0 of this sample; obstacles split over the 4 lanes
    const float px = __shfl(v[0], nn, 64), py = __shfl(v[1], nn, 64), pz = __shfl(v[2], nn, 64);
    const float4 *ob = reinterpret_cast<const float4 *>(sObs);
    const float pos[3] = {px, py, pz};
    const float xx = QuadrotorSys::scaled_sq(p, pos);   // the obstacles are scaled by p.obs_scale
    float bar = 0.f;
    for (int j = q; j < p.n_obs; j += 4) {
      const float pen = fmaxf(0.f, QuadrotorSys::barrier_arg(ob[j], pos, xx));
      bar = fmaf(pen, pen, bar);
    }
    bar += __shfl_xor(bar, 16, 64);
    bar += __shfl_xor(bar, 32, 64);
    float lr = 0.f;
    if (q == 3) {
      float quad = 0.f, lin = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) t += a.Mq[r * 4 + j] * du[j];
        quad += du[r] * t;
        lin += sRU[i * 4 + r] * du[r];
      }
      lr = quad + lin + sC[i];
    }
    lr = __shfl(lr, 48 + nn, 64);
    const float dx = px - p.goal[0], dy = py - p.goal[1], dz = pz - p.goal[2];
    const float qt = (p.wg * (dx * dx + dy * dy + dz * dz) + p.wo_s * bar) + lr;
    S += (double)qt;
  }
  if (!isfinite(S)) S = __builtin_inf();
  const bool valid = q == 0 && k < a.K;
  if (valid) a.S[k] = S;
  const double bm = block_min(valid ? S : __builtin_inf(), red);
  if (threadIdx.x == 0) a.blk_min[blockIdx.x] = bm;
}

}  // namespace mppi

// ===================================================================== host side
using namespace mppi;

#define HIP_TRY(call)                                 \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return hip_fail(_e, #call); \
  } while (0)

struct mppi_mlp {
  int device = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // FP32 params, grads, Adam moments
  __bf16 *frag = nullptr;             // training fragments, packed from p after every update
  double *stats = nullptr;
  int64_t adam_t = 0;
  float *Z = nullptr, *D = nullptr;   // dataset
  int64_t n = 0;
  // batch scratch (capacity cap)
  int cap = 0;
  char *scratch = nullptr;
  hipStream_t stream = nullptr;
  // training: the Adam step count and step size the captured steps read (device), the
  // minibatch order and per-step losses (device, capacities in elements), and one captured
  // graph of a whole call per (steps, batch), valid while these buffers stay in place
  float *d_lr = nullptr;
  float *d_corr = nullptr;            // [2 steps] Adam bias corrections 1 - beta^t of the call
  int32_t *d_order = nullptr;
  int64_t order_cap = 0;
  double *d_losses = nullptr;
  int64_t loss_cap = 0;
  float h_lr = 0.f;
  std::vector<float> h_corr;
  std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
};

namespace {

// Per-minibatch buffers (capacity B): direct inputs, forward outputs, the blocks' partials.
struct BatchBufs {
  __bf16 *Xh;                      // [B][16]
  float *Tn, *Yc;                  // [B][12]
  float *P;                        // [blocks][kNParams]
  double *Pb, *Pl, *loss;          // [blocks][kNBias], [blocks], [1]
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
inline int train_blocks(int B) { return (B + kTrainSamples - 1) / kTrainSamples; }

BatchBufs carve(char *base, int B, size_t *total = nullptr) {
  BatchBufs b;
  size_t o = 0;
  auto take = [&](size_t bytes) { char *r = base + o; o = al256(o + bytes); return r; };
  const int nbk = train_blocks(B);
  b.Xh = (__bf16 *)take((size_t)B * 16 * 2);
  b.Tn = (float *)take((size_t)B * kOut * 4);
  b.Yc = (float *)take((size_t)B * kOut * 4);
  b.P = (float *)take((size_t)nbk * kNParams * 4);
  b.Pb = (double *)take((size_t)nbk * kNBias * 8);
  b.Pl = (double *)take((size_t)nbk * 8);
  b.loss = (double *)take(8);
  if (total) *total = o;
  return b;
}

void clear_graphs(mppi_mlp *m) {
  for (auto &kv : m->graphs) (void)hipGraphExecDestroy(kv.second);
  m->graphs.clear();
}

int ensure_cap(mppi_mlp *m, int B) {
  if (B <= m->cap) return MPPI_OK;
  (void)hipStreamSynchronize(m->stream);
  clear_graphs(m);
  if (m->scratch) (void)hipFree(m->scratch);
  m->scratch = nullptr;
  m->cap = 0;
  size_t bytes = 0;
  (void)carve(nullptr, B, &bytes);
  HIP_TRY(hipMalloc((void **)&m->scratch, bytes));
  m->cap = B;
  return MPPI_OK;
}

inline int nb(long n, int t = 256) { return (int)((n + t - 1) / t); }

int prepare_train_kernel() {
  static bool done = false;
  if (!done) {
    HIP_TRY(hipFuncSetAttribute((const void *)train_step_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kTrainLds));
    done = true;
  }
  return MPPI_OK;
}

void repack(mppi_mlp *m) {
  hipLaunchKernelGGL(pack_train_kernel, dim3(nb(kTrainFrags * 64 * 8)), dim3(256), 0, m->stream, m->p, m->frag);
}

TrainArgs train_args(mppi_mlp *m, const BatchBufs &b, int B, const int *order, int backward) {
  TrainArgs t;
  std::memset(&t, 0, sizeof(t));
  t.Z = m->Z; t.D = m->D; t.order = order; t.Xh = b.Xh; t.Tn = b.Tn; t.stats = m->stats; t.p = m->p;
  t.frag = (const bf16x8 *)m->frag; t.B = B; t.backward = backward; t.Yc = b.Yc; t.P = b.P; t.Pb = b.Pb; t.Pl = b.Pl;
  return t;
}

// One minibatch on stream st: the fused forward/backward, then the reduction (with update,
// Adam with the call's bias corrections and the new weights into the fragments).
void step(mppi_mlp *m, const BatchBufs &b, int B, const int *order, bool update, int step_no, hipStream_t st,
          double *loss_out) {
  const TrainArgs t = train_args(m, b, B, order, 1);
  hipLaunchKernelGGL(train_step_kernel, dim3(train_blocks(B)), dim3(256), kTrainLds, st, t);
  hipLaunchKernelGGL(train_reduce_kernel, dim3(nb(4L * kNParams)), dim3(256), 0, st, b.P, b.Pb, b.Pl, train_blocks(B),
                     B, m->g, m->p, m->m, m->v, update ? 1 : 0, m->d_corr, step_no, m->d_lr, m->frag, loss_out);
}

int check_mlp(mppi_mlp *m) {
  if (!m) return fail(MPPI_EINVAL, "mlp is NULL");
  HIP_TRY(hipSetDevice(m->device));
  return MPPI_OK;
}

QuadrotorSys::Params quad_params_dev(const mppi_quadrotor_params *q) {
  QuadrotorSys::Params qp;
  std::memset(&qp, 0, sizeof(qp));
  qp.m_inv = (float)(1.0 / q->mass); qp.dm_inv = 1.0 / q->mass;
  qp.g = (float)q->gravity; qp.dg = q->gravity;
  qp.arm = (float)q->arm; qp.darm = q->arm;
  qp.kap = (float)q->yaw_coef; qp.dkap = q->yaw_coef;
  for (int i = 0; i < 3; ++i) {
    qp.J[i] = (float)q->inertia[i]; qp.dJ[i] = q->inertia[i];
    qp.Jinv[i] = (float)(1.0 / q->inertia[i]); qp.dJinv[i] = 1.0 / q->inertia[i];
  }
  return qp;
}

}  // namespace

extern "C" int mppi_mlp_create(int32_t device, const float *params, mppi_mlp **out) {
  if (!params || !out) return fail(MPPI_EINVAL, "params and out must be non-NULL");
  *out = nullptr;
  for (int i = 0; i < kNParams; ++i)
    if (!std::isfinite(params[i])) return fail(MPPI_EINVAL, "params has non-finite entries");
  int rc = set_device(device);
  if (rc) return rc;
  auto *m = new mppi_mlp();
  m->device = device;
  int rc2 = prepare_train_kernel();
  if (rc2) { delete m; return rc2; }
  hipError_t e = hipMalloc((void **)&m->p, kNParams * 4 * 4);
  if (e == hipSuccess) e = hipMalloc((void **)&m->frag, (size_t)kTrainFrags * 64 * 16);
  if (e == hipSuccess) e = hipMalloc((void **)&m->stats, MPPI_MLP_STATS * 8 + 256);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
  if (e != hipSuccess) { mppi_mlp_destroy(m); return fail(MPPI_ENOMEM, "mlp allocation: %s", hipGetErrorString(e)); }
  m->g = m->p + kNParams;
  m->m = m->g + kNParams;
  m->v = m->m + kNParams;
  m->d_lr = (float *)(m->stats + MPPI_MLP_STATS);
  std::vector<float> zeros(3 * kNParams, 0.f);
  std::vector<double> st(MPPI_MLP_STATS, 0.0);
  for (int i = 16; i < 32; ++i) st[i] = 1.0;
  for (int i = 44; i < 56; ++i) st[i] = 1.0;
  e = hipMemcpy(m->p, params, kNParams * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->g, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stats, st.data(), st.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) { mppi_mlp_destroy(m); return hip_fail(e, "mlp upload"); }
  repack(m);
  e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) { mppi_mlp_destroy(m); return hip_fail(e, "mlp init"); }
  *out = m;
  return MPPI_OK;
}

extern "C" int mppi_mlp_destroy(mppi_mlp *m) {
  if (!m) return MPPI_OK;
  (void)hipSetDevice(m->device);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  if (m->p) (void)hipFree(m->p);
  clear_graphs(m);
  if (m->frag) (void)hipFree(m->frag);
  if (m->d_order) (void)hipFree(m->d_order);
  if (m->d_losses) (void)hipFree(m->d_losses);
  if (m->stats) (void)hipFree(m->stats);
  if (m->Z) (void)hipFree(m->Z);
  if (m->scratch) (void)hipFree(m->scratch);
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
  return MPPI_OK;
}

extern "C" int mppi_mlp_set_dataset(mppi_mlp *m, const mppi_quadrotor_params *quad, double dt, const double *x,
                                    const double *u, int64_t n) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!quad || !x || !u || n < 1 || n > (int64_t)1 << 26 || !(dt > 0)) return fail(MPPI_EINVAL, "bad dataset arguments");
  if (!(quad->mass > 0) || !(quad->inertia[0] > 0) || !(quad->inertia[1] > 0) || !(quad->inertia[2] > 0))
    return fail(MPPI_EINVAL, "quadrotor mass and inertia must be > 0");
  HIP_TRY(hipStreamSynchronize(m->stream));
  clear_graphs(m);                         // captured training steps hold the old dataset's address
  if (m->Z) (void)hipFree(m->Z);
  m->Z = nullptr;
  m->n = 0;
  HIP_TRY(hipMalloc((void **)&m->Z, (size_t)n * 28 * 4));
  m->D = m->Z + (size_t)n * 16;
  double *dx = nullptr, *du = nullptr;
  HIP_TRY(hipMalloc((void **)&dx, (size_t)n * 16 * 8));
  du = dx + (size_t)n * 12;
  hipError_t e = hipMemcpy(dx, x, (size_t)n * 12 * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(du, u, (size_t)n * 4 * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(dataset_kernel, dim3(nb(n)), dim3(256), 0, m->stream, dx, du, (long)n, dt, quad_params_dev(quad),
                       m->Z, m->D);
    hipLaunchKernelGGL(moments_kernel, dim3(28), dim3(256), 0, m->stream, m->Z, m->D, (long)n, m->stats);
    e = hipStreamSynchronize(m->stream);
  }
  (void)hipFree(dx);
  if (e != hipSuccess) return hip_fail(e, "dataset");
  m->n = n;
  return MPPI_OK;
}

extern "C" int mppi_mlp_get_targets(mppi_mlp *m, double *out, int64_t n) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!out || n != m->n) return fail(MPPI_EINVAL, "targets: n must equal the dataset size");
  std::vector<float> f((size_t)n * 12);
  HIP_TRY(hipMemcpy(f.data(), m->D, f.size() * 4, hipMemcpyDeviceToHost));
  for (size_t i = 0; i < f.size(); ++i) out[i] = f[i];
  return MPPI_OK;
}

extern "C" int mppi_mlp_set_stats(mppi_mlp *m, const double *stats) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!stats) return fail(MPPI_EINVAL, "stats is NULL");
  for (int i = 0; i < MPPI_MLP_STATS; ++i)
    if (!std::isfinite(stats[i]) || ((i >= 16 && i < 32) || i >= 44 ? !(stats[i] > 0) : false))
      return fail(MPPI_EINVAL, "stats: non-finite entry or non-positive deviation");
  HIP_TRY(hipMemcpy(m->stats, stats, MPPI_MLP_STATS * 8, hipMemcpyHostToDevice));
  return MPPI_OK;
}

extern "C" int mppi_mlp_get_stats(mppi_mlp *m, double *stats) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!stats) return fail(MPPI_EINVAL, "stats is NULL");
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(stats, m->stats, MPPI_MLP_STATS * 8, hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" int mppi_mlp_get_params(mppi_mlp *m, float *params) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!params) return fail(MPPI_EINVAL, "params is NULL");
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(params, m->p, kNParams * 4, hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" int mppi_mlp_set_params(mppi_mlp *m, const float *params) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!params) return fail(MPPI_EINVAL, "params is NULL");
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(m->p, params, kNParams * 4, hipMemcpyHostToDevice));
  repack(m);
  HIP_TRY(hipStreamSynchronize(m->stream));
  return MPPI_OK;
}

extern "C" int mppi_mlp_train(mppi_mlp *m, const int32_t *order, int64_t n_order, int32_t batch, double lr,
                              double *losses) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!order || batch < 1 || batch > 65536 || n_order < batch || !(lr > 0)) return fail(MPPI_EINVAL, "bad training arguments");
  if (m->n < 1) return fail(MPPI_EINVAL, "no dataset");
  for (int64_t i = 0; i < n_order; ++i)
    if (order[i] < 0 || order[i] >= m->n) return fail(MPPI_EINVAL, "order[%lld] outside the dataset", (long long)i);
  rc = ensure_cap(m, batch);
  if (rc) return rc;
  const BatchBufs b = carve(m->scratch, batch);
  const int64_t steps = n_order / batch;
  if (steps * batch > m->order_cap || steps > m->loss_cap) {
    HIP_TRY(hipStreamSynchronize(m->stream));
    clear_graphs(m);
    if (steps * batch > m->order_cap) {
      if (m->d_order) (void)hipFree(m->d_order);
      m->d_order = nullptr;
      m->order_cap = 0;
      HIP_TRY(hipMalloc((void **)&m->d_order, (size_t)steps * batch * 4));
      m->order_cap = steps * batch;
    }
    if (steps > m->loss_cap) {
      if (m->d_losses) (void)hipFree(m->d_losses);
      m->d_losses = nullptr;
      m->d_corr = nullptr;
      m->loss_cap = 0;
      HIP_TRY(hipMalloc((void **)&m->d_losses, (size_t)steps * 16));   // losses, then the corrections
      m->d_corr = (float *)(m->d_losses + steps);
      m->loss_cap = steps;
    }
  }
  // the call's inputs on the stream ahead of its steps: the order, the Adam count, the step size
  m->h_lr = (float)lr;
  m->h_corr.resize((size_t)2 * steps);
  for (int64_t s = 0; s < steps; ++s) {
    const double t = (double)(m->adam_t + s + 1);
    m->h_corr[2 * s] = (float)(1.0 - std::pow(0.9, t));
    m->h_corr[2 * s + 1] = (float)(1.0 - std::pow(0.999, t));
  }
  HIP_TRY(hipMemcpyAsync(m->d_order, order, (size_t)steps * batch * 4, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipMemcpyAsync(m->d_corr, m->h_corr.data(), (size_t)steps * 8, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipMemcpyAsync(m->d_lr, &m->h_lr, 4, hipMemcpyHostToDevice, m->stream));
  // all steps of the call as one captured graph, kept for the next call of the same shape
  auto key = std::make_pair(steps, (int)batch);
  auto it = m->graphs.find(key);
  if (it == m->graphs.end()) {
    hipGraph_t gr = nullptr;
    hipGraphExec_t ge = nullptr;
    HIP_TRY(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    for (int64_t s = 0; s < steps; ++s) step(m, b, batch, m->d_order + s * batch, true, (int)s, m->stream, m->d_losses + s);
    ce = hipGetLastError();
    hipError_t e = hipStreamEndCapture(m->stream, &gr);
    if (ce != hipSuccess || e != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return hip_fail(ce != hipSuccess ? ce : e, "training capture");
    }
    e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return hip_fail(e, "training graph");
    it = m->graphs.emplace(key, ge).first;
  }
  hipError_t e = hipGraphLaunch(it->second, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess && losses) e = hipMemcpy(losses, m->d_losses, (size_t)steps * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "training");
  m->adam_t += steps;
  return MPPI_OK;
}

extern "C" int mppi_mlp_loss_grads(mppi_mlp *m, const double *zn, const double *tn, int32_t B, double *loss, float *grads) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!zn || !tn || B < 1 || B > 65536) return fail(MPPI_EINVAL, "bad loss_grads arguments");
  rc = ensure_cap(m, B);
  if (rc) return rc;
  const BatchBufs b = carve(m->scratch, B);
  std::vector<__bf16> xh((size_t)B * 16);
  std::vector<float> t((size_t)B * 12);
  for (size_t i = 0; i < xh.size(); ++i) xh[i] = (__bf16)(float)zn[i];
  for (size_t i = 0; i < t.size(); ++i) t[i] = (float)tn[i];
  HIP_TRY(hipMemcpyAsync(b.Xh, xh.data(), xh.size() * 2, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipMemcpyAsync(b.Tn, t.data(), t.size() * 4, hipMemcpyHostToDevice, m->stream));
  step(m, b, B, nullptr, false, 0, m->stream, b.loss);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(m->stream));
  if (loss) HIP_TRY(hipMemcpy(loss, b.loss, 8, hipMemcpyDeviceToHost));
  if (grads) HIP_TRY(hipMemcpy(grads, m->g, kNParams * 4, hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" int mppi_mlp_forward(mppi_mlp *m, const double *x, const double *u, int32_t B, double *dx) {
  int rc = check_mlp(m);
  if (rc) return rc;
  if (!x || !u || !dx || B < 1 || B > 65536) return fail(MPPI_EINVAL, "bad forward arguments");
  rc = ensure_cap(m, B);
  if (rc) return rc;
  const BatchBufs b = carve(m->scratch, B);
  double *dev = nullptr;
  HIP_TRY(hipMalloc((void **)&dev, (size_t)B * 28 * 8));
  double *dxd = dev + (size_t)B * 16;
  hipError_t e = hipMemcpyAsync(dev, x, (size_t)B * 12 * 8, hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dev + (size_t)B * 12, u, (size_t)B * 4 * 8, hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(std_inputs_kernel, dim3(nb((long)B * 16)), dim3(256), 0, m->stream, dev, dev + (size_t)B * 12,
                       m->stats, B, b.Xh);
    const TrainArgs t = train_args(m, b, B, nullptr, 0);
    hipLaunchKernelGGL(train_step_kernel, dim3(train_blocks(B)), dim3(256), kTrainLds, m->stream, t);
    hipLaunchKernelGGL(dx_out_kernel, dim3(nb((long)B * kOut)), dim3(256), 0, m->stream, b.Yc, m->p + kOffB3, m->stats, B, dxd);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess) e = hipMemcpy(dx, dxd, (size_t)B * 12 * 8, hipMemcpyDeviceToHost);
  (void)hipFree(dev);
  if (e != hipSuccess) return hip_fail(e, "mlp forward");
  return MPPI_OK;
}

// ------------------------------------------------------------- controller hooks
namespace mppi {

struct MlpState {
  bf16x8 *frag = nullptr;   // packed rollout fragments
  float *params = nullptr;  // FP32 copy (biases)
  double *stats = nullptr;
};

uint64_t extra_workspace_bytes(const mppi_config *) { return 0; }

int init_extra(mppi_ctx *c, const mppi_config *cfg) {
  if (cfg->system != MPPI_SYS_QUADROTOR_MLP) return MPPI_OK;
  const mppi_mlp *src = ((const mppi_quadrotor_mlp_params *)cfg->params)->mlp;
  if (src->device != cfg->device) return fail(MPPI_EINVAL, "the mlp lives on device %d, the controller on %d", src->device, cfg->device);
  auto *st = new MlpState();
  c->mlp = st;
  hipError_t e = hipMalloc((void **)&st->frag, (size_t)kFrags * 64 * 16 + kNParams * 4 + MPPI_MLP_STATS * 8);
  if (e != hipSuccess) return fail(MPPI_ENOMEM, "mlp rollout buffers: %s", hipGetErrorString(e));
  st->params = (float *)((char *)st->frag + (size_t)kFrags * 64 * 16);
  st->stats = (double *)(st->params + kNParams);
  e = hipStreamSynchronize(src->stream);
  if (e == hipSuccess) e = hipMemcpy(st->params, src->p, kNParams * 4, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(st->stats, src->stats, MPPI_MLP_STATS * 8, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pack_rollout_kernel, dim3(nb(kFrags * 64 * 8)), dim3(256), 0, 0, st->params, (__bf16 *)st->frag);
    e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) return hip_fail(e, "mlp rollout pack");
  return MPPI_OK;
}

void destroy_extra(mppi_ctx *c) {
  if (!c->mlp) return;
  if (c->mlp->frag) (void)hipFree(c->mlp->frag);
  delete c->mlp;
  c->mlp = nullptr;
}

size_t mlp_rollout_lds(const mppi_ctx *c) {
  const int T = c->cfg.T;
  size_t fl = (size_t)8 * T + ((T + 3) & ~3);
  fl = (fl + 3) & ~size_t(3);
  return (fl + (size_t)QuadrotorSys::stage_floats(c->quad.n_obs, 0)) * 4;
}

int prepare_mlp_rollout(mppi_ctx *c) {
  const size_t lds = mlp_rollout_lds(c);
  if (lds > 160 * 1024 - 64) return fail(MPPI_EINVAL, "mlp rollout needs %zu B of LDS (T too large)", lds);
  HIP_TRY(hipFuncSetAttribute((const void *)mlp_rollout_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return MPPI_OK;
}

int launch_mlp_rollout(mppi_ctx *c, const IterArgs &a, hipStream_t s) {
  MlpRollArgs m{c->mlp->frag, c->mlp->params, c->mlp->stats};
  IterArgs a_arg = a;
  QuadrotorSys::Params p_arg = c->quad;
  void *args[] = {(void *)&a_arg, (void *)&p_arg, (void *)&m};
  return timed_launch(c, 0, (const void *)mlp_rollout_kernel, dim3(c->L.n_roll_blocks), dim3(kBlock), args,
                      mlp_rollout_lds(c), s);
}

}  // namespace mppi
