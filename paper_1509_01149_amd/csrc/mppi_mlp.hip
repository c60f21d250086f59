// Learned dynamics on BF16 MFMA (gfx950 v_mfma_f32_16x16x32_bf16): training kernels
// (generic strided GEMM, bias + tanh, loss, tanh backward, bias gradients, Adam) and the
// fused MPPI rollout whose network weights stay in registers for the whole horizon.
// Contract: include/mppi.h, "Learned dynamics".
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
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

// ------------------------------------------------------------------ generic GEMM
// C[m][n] = sum_k A(m, k) B(k, n) over bf16 operands addressed by strides, FP32 result.
// Block = 4 waves, each wave one 16 x 16 tile of C; K advances 32 per MFMA.  Split K:
// block z covers k in [z k_chunk, (z + 1) k_chunk) and, when P is given, writes its
// partial tile to P[z] (dense M x N); reduce_splits_kernel then sums the splits in order.
// An operand whose k stride is 1 is read eight elements (16 bytes) at a time.
static __global__ __launch_bounds__(256) void gemm_bf16_kernel(const __bf16 *__restrict__ A, long sam, long sak,
                                                               const __bf16 *__restrict__ B, long sbk, long sbn,
                                                               float *__restrict__ C, long scm, long scn, int M,
                                                               int N, int K, int k_chunk, float *__restrict__ P) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int m0 = blockIdx.y * 32 + (w >> 1) * 16, n0 = blockIdx.x * 32 + (w & 1) * 16;
  const int row = l & 15, kg = l >> 4;
  const int kb = blockIdx.z * k_chunk, ke = min(K, kb + k_chunk);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  const __bf16 z = to_bf16(0.f);
  const bool a_row = m0 + row < M, b_row = n0 + row < N;
  // 16-byte vector reads need k contiguous and every row start 16-byte aligned
  const bool a_vec = sak == 1 && (sam & 7) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
  const bool b_vec = sbk == 1 && (sbn & 7) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const int k8 = k0 + 8 * kg;
    bf16x8 a, b;
    if (a_vec && a_row && k8 + 8 <= ke) {
      a = *reinterpret_cast<const bf16x8 *>(A + (long)(m0 + row) * sam + k8);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = (a_row && k8 + e < ke) ? A[(long)(m0 + row) * sam + (long)(k8 + e) * sak] : z;
    }
    if (b_vec && b_row && k8 + 8 <= ke) {
      b = *reinterpret_cast<const bf16x8 *>(B + (long)(n0 + row) * sbn + k8);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) b[e] = (b_row && k8 + e < ke) ? B[(long)(k8 + e) * sbk + (long)(n0 + row) * sbn] : z;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + 4 * kg + r, n = n0 + row;
    if (m < M && n < N) {
      if (P) P[((long)blockIdx.z * M + m) * N + n] = acc[r];
      else C[(long)m * scm + (long)n * scn] = acc[r];
    }
  }
}

// C[m][n] = sum over the splits z = 0, 1, ... of P[z][m][n], in that order.
static __global__ void reduce_splits_kernel(const float *__restrict__ P, int splits, int M, int N, float *C, long scm,
                                            long scn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  float s = 0.f;
  constexpr int kBatch = 16;                        // loads in flight per thread
  for (int z0 = 0; z0 < splits; z0 += kBatch) {
    float v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) v[j] = z0 + j < splits ? P[(long)(z0 + j) * M * N + i] : 0.f;
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (z0 + j < splits) s += v[j];
  }
  C[(long)(i / N) * scm + (long)(i % N) * scn] = s;
}

// ------------------------------------------------------------ elementwise kernels
// Standardised minibatch: X = (Z[idx] - mu) / sd -> bf16 [B][16]; T = (D[idx] - mu) / sd [B][12].
static __global__ void gather_kernel(const float *Z, const float *D, const int *order, const double *stats, int B,
                                     __bf16 *Xh, float *Tn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * 28) return;
  const int r = i / 28, c = i - r * 28;
  const long s = order[r];
  if (c < 16) Xh[r * 16 + c] = to_bf16((float)(((double)Z[s * 16 + c] - stats[c]) / stats[16 + c]));
  else Tn[r * 12 + (c - 16)] = (float)(((double)D[s * 12 + (c - 16)] - stats[32 + c - 16]) / stats[44 + c - 16]);
}

// H = tanh(Zc + b) (FP32 and bf16 copies), Zc [B][128].
static __global__ void bias_tanh_kernel(const float *Zc, const float *b, float *Hf, __bf16 *Hh, int total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float h = tanh_f(Zc[i] + b[i & (kH - 1)]);
  Hf[i] = h;
  Hh[i] = to_bf16(h);
}

// Y = Yc + b3; dY = 2 (Y - T) / (B 12) (FP32 for the bias gradient, bf16 for the products);
// per-block FP64 partial sums of (Y - T)^2 in a fixed order.
static __global__ __launch_bounds__(256) void loss_grad_kernel(const float *Yc, const float *b3, const float *Tn,
                                                               int B, float *dY, __bf16 *dYh, double *loss_part) {
  __shared__ double red[4];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (i < B * kOut) {
    const float d = Yc[i] + b3[i % kOut] - Tn[i];
    const float g = 2.f * d / (float)(B * kOut);
    dY[i] = g;
    dYh[i] = to_bf16(g);
    sq = (double)d * (double)d;
  }
  const double s = block_sum(sq, red);
  if (threadIdx.x == 0) loss_part[blockIdx.x] = s;
}

static __global__ void loss_finish_kernel(const double *loss_part, int nparts, int B, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  *out = ordered_sum(loss_part, 1, nparts) / (double)(B * kOut);   // in order, loads batched
}

// dZ = dH (1 - H^2) (FP32 and bf16).
static __global__ void tanh_bwd_kernel(const float *dH, const float *Hf, float *dZ, __bf16 *dZh, int total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float h = Hf[i];
  const float g = dH[i] * (1.f - h * h);
  dZ[i] = g;
  dZh[i] = to_bf16(g);
}

// out[c] = sum_r X[r][c] over B rows, fixed order (strided partials, then a block tree).
static __global__ __launch_bounds__(256) void colsum_kernel(const float *X, int B, int ncol, float *out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  constexpr int kBatch = 8;                         // loads in flight per thread
  for (int r0 = threadIdx.x; r0 < B; r0 += 256 * kBatch) {
    float v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) v[j] = r0 + 256 * j < B ? X[(long)(r0 + 256 * j) * ncol + c] : 0.f;
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (r0 + 256 * j < B) s += (double)v[j];
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) out[c] = (float)t;
}

// Adam on the FP32 parameters; refresh the bf16 copies of the weights.
static __global__ void adam_kernel(float *p, const float *g, float *m, float *v, int n, float lr, float c1,
                                   float c2, __bf16 *W1h, __bf16 *W2h, __bf16 *W3h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  p[i] = pi;
  if (i < kOffB1) W1h[i - kOffW1] = to_bf16(pi);
  else if (i >= kOffW2 && i < kOffB2) W2h[i - kOffW2] = to_bf16(pi);
  else if (i >= kOffW3 && i < kOffB3) W3h[i - kOffW3] = to_bf16(pi);
}

static __global__ void to_bf16_kernel(const float *p, __bf16 *W1h, __bf16 *W2h, __bf16 *W3h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNParams) return;
  if (i < kOffB1) W1h[i - kOffW1] = to_bf16(p[i]);
  else if (i >= kOffW2 && i < kOffB2) W2h[i - kOffW2] = to_bf16(p[i]);
  else if (i >= kOffW3 && i < kOffB3) W3h[i - kOffW3] = to_bf16(p[i]);
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
    float bar = 0.f;
    for (int j = q; j < p.n_obs; j += 4) {
      const float4 o = ob[j];
      const float ex = px - o.x, ey = py - o.y, ez = pz - o.z;
      const float pen = fmaxf(0.f, o.w - (ex * ex + ey * ey + ez * ez));
      bar += pen * pen;
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
    const float qt = (p.wg * (dx * dx + dy * dy + dz * dz) + p.wo * bar) + lr;
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
  __bf16 *W1h = nullptr, *W2h = nullptr, *W3h = nullptr;
  double *stats = nullptr;
  int64_t adam_t = 0;
  float *Z = nullptr, *D = nullptr;   // dataset
  int64_t n = 0;
  // batch scratch (capacity cap)
  int cap = 0;
  char *scratch = nullptr;
  hipStream_t stream = nullptr;
};

namespace {

constexpr int kMaxSplits = 64;     // split-K partial tiles for the weight gradients
constexpr int kSplitChunk = 128;   // samples per split (a multiple of the MFMA's 32)

struct BatchBufs {
  __bf16 *Xh, *H1h, *H2h, *dYh, *dZ1h, *dZ2h;
  float *Tn, *Z1, *H1, *Z2, *H2, *Y, *dY, *dH2, *dZ2, *dH1, *dZ1;
  float *part;                     // [kMaxSplits][kH][kH]
  double *loss_part, *loss;
  int *order;
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

size_t batch_bytes(int B) {
  size_t o = 0;
  auto take = [&](size_t b) { o = al256(o + b); };
  take((size_t)B * 16 * 2);                       // Xh
  for (int i = 0; i < 2; ++i) take((size_t)B * kH * 2);   // H1h H2h
  take((size_t)B * kOut * 2);                     // dYh
  for (int i = 0; i < 2; ++i) take((size_t)B * kH * 2);   // dZ1h dZ2h
  take((size_t)B * kOut * 4);                     // Tn
  for (int i = 0; i < 4; ++i) take((size_t)B * kH * 4);   // Z1 H1 Z2 H2
  take((size_t)B * kOut * 4);                     // Y
  take((size_t)B * kOut * 4);                     // dY
  for (int i = 0; i < 4; ++i) take((size_t)B * kH * 4);   // dH2 dZ2 dH1 dZ1
  take((size_t)((B * kOut + 255) / 256 + 1) * 8);  // loss_part
  take(8);                                        // loss
  take((size_t)B * 4);                            // order
  take((size_t)kMaxSplits * kH * kH * 4);         // part
  return o;
}

BatchBufs carve(char *base, int B) {
  BatchBufs b;
  size_t o = 0;
  auto take = [&](size_t bytes) { char *r = base + o; o = al256(o + bytes); return r; };
  b.Xh = (__bf16 *)take((size_t)B * 16 * 2);
  b.H1h = (__bf16 *)take((size_t)B * kH * 2);
  b.H2h = (__bf16 *)take((size_t)B * kH * 2);
  b.dYh = (__bf16 *)take((size_t)B * kOut * 2);
  b.dZ1h = (__bf16 *)take((size_t)B * kH * 2);
  b.dZ2h = (__bf16 *)take((size_t)B * kH * 2);
  b.Tn = (float *)take((size_t)B * kOut * 4);
  b.Z1 = (float *)take((size_t)B * kH * 4);
  b.H1 = (float *)take((size_t)B * kH * 4);
  b.Z2 = (float *)take((size_t)B * kH * 4);
  b.H2 = (float *)take((size_t)B * kH * 4);
  b.Y = (float *)take((size_t)B * kOut * 4);
  b.dY = (float *)take((size_t)B * kOut * 4);
  b.dH2 = (float *)take((size_t)B * kH * 4);
  b.dZ2 = (float *)take((size_t)B * kH * 4);
  b.dH1 = (float *)take((size_t)B * kH * 4);
  b.dZ1 = (float *)take((size_t)B * kH * 4);
  b.loss_part = (double *)take((size_t)((B * kOut + 255) / 256 + 1) * 8);
  b.loss = (double *)take(8);
  b.order = (int *)take((size_t)B * 4);
  b.part = (float *)take((size_t)kMaxSplits * kH * kH * 4);
  return b;
}

int ensure_cap(mppi_mlp *m, int B) {
  if (B <= m->cap) return MPPI_OK;
  if (m->scratch) (void)hipFree(m->scratch);
  m->scratch = nullptr;
  m->cap = 0;
  HIP_TRY(hipMalloc((void **)&m->scratch, batch_bytes(B)));
  m->cap = B;
  return MPPI_OK;
}

// part: split-K scratch of kMaxSplits * M * N floats, or NULL for no split.  A long K
// (the weight gradients sum over the minibatch) is cut into kSplitChunk pieces so the
// 16 output tiles become hundreds of blocks.
void gemm(hipStream_t s, const __bf16 *A, long sam, long sak, const __bf16 *B, long sbk, long sbn, float *C, long scm,
          long scn, int M, int N, int K, float *part = nullptr) {
  const dim3 grid((N + 31) / 32, (M + 31) / 32);
  int splits = part ? (K + kSplitChunk - 1) / kSplitChunk : 1;
  if (splits > kMaxSplits) splits = kMaxSplits;
  if (splits <= 1) {
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, scm, scn, M, N, K, K,
                       (float *)nullptr);
    return;
  }
  const int chunk = ((K + splits - 1) / splits + 31) / 32 * 32;
  splits = (K + chunk - 1) / chunk;
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3(grid.x, grid.y, splits), dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, scm,
                     scn, M, N, K, chunk, part);
  hipLaunchKernelGGL(reduce_splits_kernel, dim3((M * N + 255) / 256), dim3(256), 0, s, part, splits, M, N, C, scm, scn);
}

inline int nb(long n, int t = 256) { return (int)((n + t - 1) / t); }

// Forward (and optionally backward) of one minibatch already standardised into b.Xh / b.Tn.
void fwd(mppi_mlp *m, const BatchBufs &b, int B) {
  hipStream_t s = m->stream;
  gemm(s, b.Xh, 16, 1, m->W1h, 1, 16, b.Z1, kH, 1, B, kH, kIn);
  hipLaunchKernelGGL(bias_tanh_kernel, dim3(nb((long)B * kH)), dim3(256), 0, s, b.Z1, m->p + kOffB1, b.H1, b.H1h, B * kH);
  gemm(s, b.H1h, kH, 1, m->W2h, 1, kH, b.Z2, kH, 1, B, kH, kH);
  hipLaunchKernelGGL(bias_tanh_kernel, dim3(nb((long)B * kH)), dim3(256), 0, s, b.Z2, m->p + kOffB2, b.H2, b.H2h, B * kH);
  gemm(s, b.H2h, kH, 1, m->W3h, 1, kH, b.Y, kOut, 1, B, kOut, kH);
}

void bwd(mppi_mlp *m, const BatchBufs &b, int B) {
  hipStream_t s = m->stream;
  const int nparts = nb((long)B * kOut);
  hipLaunchKernelGGL(loss_grad_kernel, dim3(nparts), dim3(256), 0, s, b.Y, m->p + kOffB3, b.Tn, B, b.dY, b.dYh,
                     b.loss_part);
  hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(64), 0, s, b.loss_part, nparts, B, b.loss);
  // data gradients
  gemm(s, b.dYh, kOut, 1, m->W3h, kH, 1, b.dH2, kH, 1, B, kH, kOut);
  hipLaunchKernelGGL(tanh_bwd_kernel, dim3(nb((long)B * kH)), dim3(256), 0, s, b.dH2, b.H2, b.dZ2, b.dZ2h, B * kH);
  gemm(s, b.dZ2h, kH, 1, m->W2h, kH, 1, b.dH1, kH, 1, B, kH, kH);
  hipLaunchKernelGGL(tanh_bwd_kernel, dim3(nb((long)B * kH)), dim3(256), 0, s, b.dH1, b.H1, b.dZ1, b.dZ1h, B * kH);
  // weight gradients: sum over the batch (k = sample)
  gemm(s, b.dYh, 1, kOut, b.H2h, kH, 1, m->g + kOffW3, kH, 1, kOut, kH, B, b.part);
  gemm(s, b.dZ2h, 1, kH, b.H1h, kH, 1, m->g + kOffW2, kH, 1, kH, kH, B, b.part);
  gemm(s, b.dZ1h, 1, kH, b.Xh, 16, 1, m->g + kOffW1, kIn, 1, kH, kIn, B, b.part);
  hipLaunchKernelGGL(colsum_kernel, dim3(kOut), dim3(256), 0, s, b.dY, B, kOut, m->g + kOffB3);
  hipLaunchKernelGGL(colsum_kernel, dim3(kH), dim3(256), 0, s, b.dZ2, B, kH, m->g + kOffB2);
  hipLaunchKernelGGL(colsum_kernel, dim3(kH), dim3(256), 0, s, b.dZ1, B, kH, m->g + kOffB1);
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
  hipError_t e = hipMalloc((void **)&m->p, kNParams * 4 * 4);
  if (e == hipSuccess) e = hipMalloc((void **)&m->W1h, (size_t)(kH * kIn + kH * kH + kOut * kH) * 2);
  if (e == hipSuccess) e = hipMalloc((void **)&m->stats, MPPI_MLP_STATS * 8);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
  if (e != hipSuccess) { mppi_mlp_destroy(m); return fail(MPPI_ENOMEM, "mlp allocation: %s", hipGetErrorString(e)); }
  m->g = m->p + kNParams;
  m->m = m->g + kNParams;
  m->v = m->m + kNParams;
  m->W2h = m->W1h + kH * kIn;
  m->W3h = m->W2h + kH * kH;
  std::vector<float> zeros(3 * kNParams, 0.f);
  std::vector<double> st(MPPI_MLP_STATS, 0.0);
  for (int i = 16; i < 32; ++i) st[i] = 1.0;
  for (int i = 44; i < 56; ++i) st[i] = 1.0;
  e = hipMemcpy(m->p, params, kNParams * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->g, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stats, st.data(), st.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) { mppi_mlp_destroy(m); return hip_fail(e, "mlp upload"); }
  hipLaunchKernelGGL(to_bf16_kernel, dim3(nb(kNParams)), dim3(256), 0, m->stream, m->p, m->W1h, m->W2h, m->W3h);
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
  if (m->W1h) (void)hipFree(m->W1h);
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
  hipLaunchKernelGGL(to_bf16_kernel, dim3(nb(kNParams)), dim3(256), 0, m->stream, m->p, m->W1h, m->W2h, m->W3h);
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
  int32_t *d_order = nullptr;
  double *d_losses = nullptr;
  HIP_TRY(hipMalloc((void **)&d_order, (size_t)steps * batch * 4));
  hipError_t e = hipMalloc((void **)&d_losses, (size_t)steps * 8);
  if (e == hipSuccess) e = hipMemcpyAsync(d_order, order, (size_t)steps * batch * 4, hipMemcpyHostToDevice, m->stream);
  for (int64_t s = 0; s < steps && e == hipSuccess; ++s) {
    hipLaunchKernelGGL(gather_kernel, dim3(nb((long)batch * 28)), dim3(256), 0, m->stream, m->Z, m->D,
                       d_order + s * batch, m->stats, batch, b.Xh, b.Tn);
    fwd(m, b, batch);
    bwd(m, b, batch);
    m->adam_t += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)m->adam_t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)m->adam_t));
    hipLaunchKernelGGL(adam_kernel, dim3(nb(kNParams)), dim3(256), 0, m->stream, m->p, m->g, m->m, m->v, kNParams,
                       (float)lr, c1, c2, m->W1h, m->W2h, m->W3h);
    e = hipMemcpyAsync(d_losses + s, b.loss, 8, hipMemcpyDeviceToDevice, m->stream);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess && losses) e = hipMemcpy(losses, d_losses, (size_t)steps * 8, hipMemcpyDeviceToHost);
  (void)hipFree(d_order);
  if (d_losses) (void)hipFree(d_losses);
  if (e != hipSuccess) return hip_fail(e, "training");
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
  fwd(m, b, B);
  bwd(m, b, B);
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
    fwd(m, b, B);
    hipLaunchKernelGGL(dx_out_kernel, dim3(nb((long)B * kOut)), dim3(256), 0, m->stream, b.Y, m->p + kOffB3, m->stats, B, dxd);
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
