// The MPPI iteration as three kernels (paper: Algorithm 1 with the likelihood-ratio
// running cost and update law of Section III-C):
//
//   rollout<Sys>  one lane per sample: draw the perturbations from Philox in registers,
//                 Euler-step the dynamics over the horizon, accumulate the path cost
//                 S_k = sum_i [q(x_{i+1}) + (1 - 1/nu)/2 du'R du + u'R du + u'R u/2] + phi
//                 (FP32 arithmetic per step, FP64 running sum), write S_k and the block
//                 minimum.
//   update        2-D grid over (sample chunk, noise group): rho = min_k S_k,
//                 w_k = exp(-(S_k - rho)/lambda) in FP64, regenerate the same normals and
//                 accumulate sum_k w_k eps_k in FP64; fixed-order reductions, no atomics.
//   finalize      one block: eta = sum_k w_k, dU = sqrt(nu) L (sum_k w_k eps_k) / eta,
//                 U += dU (FP64 master, FP32 copy for the next rollout); on the last
//                 iteration of a control step emit u0 and apply the warm shift.
#pragma once
#include "mppi_systems.h"

namespace mppi {

constexpr int kUpdGroups = 16;                       // noise groups per update block
constexpr int kUpdStrips = kBlock / kUpdGroups;      // sample strips per update block
constexpr int kUpdChunk = 256;                       // samples per update block
constexpr int kUpdPerThread = kUpdChunk / kUpdStrips;

struct IterArgs {
  const double *x0;        // [n]
  const float *U32;        // [T*m] FP32 copy of the nominal sequence
  double *S;               // [K] path costs
  double *blk_min;         // [n_roll_blocks]
  const uint64_t *iter;    // iteration counter (keys the noise)
  double *part;            // [n_kc][G*4] partial sums of w*eps
  double *eta_part;        // [n_kc]
  uint32_t key0, key1;
  int n;                   // state dimension actually present in x0 (<= Sys::N)
  int K, T, m, G;          // G = ceil(T*m/4) noise groups per sample
  int n_roll_blocks, n_kc;
  float dt;
  float lr_quad;           // (1 - 1/nu)/2
  float Ls[16];            // sqrt(nu) chol(Sigma), row-major m x m (lower)
  float R[16];             // m x m
  double inv_lambda;
};

struct FinalizeArgs {
  double *U64;             // [T*m] FP64 master
  float *U32;              // [T*m]
  const double *blk_min;
  const double *part;
  const double *eta_part;
  uint64_t *iter;
  int *flags;              // bit 0: an iteration had no finite cost
  double *dbg;             // [2 + T*m]: rho, eta, dU
  double *u0_out;          // [m]; written when emit != 0
  int T, m, G, n_roll_blocks, n_kc;
  int emit;                // last iteration of the control step: emit u0 and shift
  double Ls[16];           // sqrt(nu) chol(Sigma)
  double u_init[4];
};

// ------------------------------------------------------------------------ rollout
// One 256-sample block of one controller (`blk` indexes the controller's blocks).
// The single-controller kernel and the batched serving kernel both call this body, so a
// controller's results do not depend on what else shares the launch.
template <class Sys>
__device__ __forceinline__ void rollout_body(const IterArgs &a, const typename Sys::Params &p, const double *x0,
                                             int blk, float4 *lds4) {
  constexpr int N = Sys::N, M = Sys::M;
  constexpr int SPG = 4 / M;                        // steps per noise group
  float *sU = reinterpret_cast<float *>(lds4);      // [T*M]
  float *sRU = sU + a.T * M;                        // [T*M]  R u_i
  float *sC = sRU + a.T * M;                        // [T]    u_i'R u_i / 2
  float *sSys = sU + ((2 * a.T * M + ((a.T + 3) & ~3) + 3) & ~3);   // system staging, 16-B aligned
  __shared__ double red[4];

  const uint64_t it = *a.iter;
  for (int i = threadIdx.x; i < a.T; i += kBlock) {
    float u[M];
#pragma unroll
    for (int j = 0; j < M; ++j) u[j] = a.U32[i * M + j];
    float c = 0.f;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      float s = 0.f;
#pragma unroll
      for (int j = 0; j < M; ++j) s += a.R[r * M + j] * u[j];
      sU[i * M + r] = u[r];
      sRU[i * M + r] = s;
      c += u[r] * s;
    }
    sC[i] = 0.5f * c;
  }
  int ti = 0, tj = 0;                               // every thread computes the same origin
  Sys::stage(p, sSys, x0, &ti, &tj);
  __syncthreads();
  const StageView sv{sSys, ti, tj};

  const int k = blk * kBlock + threadIdx.x;
  float x[N];
#pragma unroll
  for (int r = 0; r < N; ++r) x[r] = r < a.n ? (float)x0[r] : 0.f;
  double S = 0.0;
  for (int g = 0; g < a.G; ++g) {
    float e[4];
    normals4((uint32_t)g, (uint32_t)k, it, a.key0, a.key1, e);
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      const int i = g * SPG + s;
      if (i < a.T) {
        float du[M], v[M], xd[N];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          float t = 0.f;
#pragma unroll
          for (int l = 0; l <= j; ++l) t += a.Ls[j * M + l] * e[s * M + l];
          du[j] = t;
          v[j] = sU[i * M + j] + t;
        }
        Sys::xdot(p, x, v, xd);
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] += a.dt * xd[r];
        float quad = 0.f, lin = 0.f;
#pragma unroll
        for (int r = 0; r < M; ++r) {
          float t = 0.f;
#pragma unroll
          for (int j = 0; j < M; ++j) t += a.R[r * M + j] * du[j];
          quad += du[r] * t;
          lin += sRU[i * M + r] * du[r];
        }
        const float qt = Sys::q(p, sv, x) + (a.lr_quad * quad + lin + sC[i]);
        S += (double)qt;
      }
    }
  }
  S += (double)Sys::phi(p, x);
  if (!isfinite(S)) S = __builtin_inf();
  const bool valid = k < a.K;
  if (valid) a.S[k] = S;
  const double bm = block_min(valid ? S : __builtin_inf(), red);
  if (threadIdx.x == 0) a.blk_min[blk] = bm;
}

template <class Sys>
__global__ __launch_bounds__(kBlock) void rollout_kernel(const IterArgs a, const typename Sys::Params p) {
  extern __shared__ float4 lds4[];
  rollout_body<Sys>(a, p, a.x0, blockIdx.x, lds4);
}

// Minimum over the rollout blocks' minima (every thread gets it).
__device__ __forceinline__ double global_min(const double *blk_min, int n, double *red) {
  double v = __builtin_inf();
  for (int b = threadIdx.x; b < n; b += kBlock) v = fmin(v, blk_min[b]);
  return block_min(v, red);
}

// ------------------------------------------------------------------------- update
// grid (n_kc, ceil(G / kUpdGroups)).  Thread t handles noise group gc*16 + t%16 for the
// samples of strip t/16 of this block's 256-sample chunk.
__device__ __forceinline__ void update_body(const IterArgs &a, int kc, int gcb) {
  __shared__ double w[kUpdChunk];
  __shared__ double acc_lds[kUpdStrips][kUpdGroups][4];
  __shared__ double red[4];
  const double rho = global_min(a.blk_min, a.n_roll_blocks, red);
  const uint64_t it = *a.iter;
  {
    const int k = kc * kUpdChunk + threadIdx.x;
    double wk = 0.0;
    if (k < a.K && rho < __builtin_inf()) {
      const double s = a.S[k];
      wk = s < __builtin_inf() ? exp(-(s - rho) * a.inv_lambda) : 0.0;
    }
    w[threadIdx.x] = wk;
    if (gcb == 0) {
      const double e = block_sum(wk, red);
      if (threadIdx.x == 0) a.eta_part[kc] = e;
    }
  }
  __syncthreads();
  const int gl = threadIdx.x % kUpdGroups, strip = threadIdx.x / kUpdGroups;
  const int g = gcb * kUpdGroups + gl;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (g < a.G) {
    for (int r = 0; r < kUpdPerThread; ++r) {
      const int kl = strip * kUpdPerThread + r;
      const double wk = w[kl];
      if (wk != 0.0) {
        float e[4];
        normals4((uint32_t)g, (uint32_t)(kc * kUpdChunk + kl), it, a.key0, a.key1, e);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = fma(wk, (double)e[c], acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) acc_lds[strip][gl][c] = acc[c];
  __syncthreads();
  if (threadIdx.x < kUpdGroups * 4) {
    const int gg = threadIdx.x / 4, c = threadIdx.x % 4;
    const int gabs = gcb * kUpdGroups + gg;
    double s = 0.0;
    for (int st = 0; st < kUpdStrips; ++st) s += acc_lds[st][gg][c];
    if (gabs < a.G) a.part[(size_t)kc * (a.G * 4) + gabs * 4 + c] = s;
  }
}

static __global__ __launch_bounds__(kBlock) void update_kernel(const IterArgs a) {
  update_body(a, blockIdx.x, blockIdx.y);
}

// ----------------------------------------------------------------------- finalize
// One block of 1024 threads; T*m <= 4096 handled in a strided loop.  Sums over the
// chunk partials run in a fixed order (c = 0, 1, ...) with their loads issued eight at
// a time, so the result is independent of timing and of the batch it runs in.
constexpr int kFinBlock = 1024;
constexpr int kMaxTM = 4096;

__device__ __forceinline__ double ordered_sum(const double *p, size_t stride, int n) {
  double s = 0.0;
  int c = 0;
  for (; c + 8 <= n; c += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = p[(size_t)(c + j) * stride];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  for (; c < n; ++c) s += p[(size_t)c * stride];
  return s;
}

// status_out (nullable): 0 when the iteration had a finite cost, -5 otherwise.
__device__ __forceinline__ void finalize_body(const FinalizeArgs &a, double *u0_out, double *status_out) {
  __shared__ double N_lds[kMaxTM];
  __shared__ double red[16];
  __shared__ double eta_s;
  const int TM = a.T * a.m;
  double v = __builtin_inf();
  for (int b = threadIdx.x; b < a.n_roll_blocks; b += kFinBlock) v = fmin(v, a.blk_min[b]);
  v = wave_min(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = v;
  if (threadIdx.x == 0) eta_s = ordered_sum(a.eta_part, 1, a.n_kc);
  for (int f = threadIdx.x; f < TM; f += kFinBlock) N_lds[f] = ordered_sum(a.part + f, (size_t)a.G * 4, a.n_kc);
  __syncthreads();
  double rho = red[0];
  for (int i = 1; i < kFinBlock / 64; ++i) rho = fmin(rho, red[i]);
  const bool ok = rho < __builtin_inf();
  const double eta = eta_s;
  const double inv_eta = ok ? 1.0 / eta : 0.0;
  for (int f = threadIdx.x; f < TM; f += kFinBlock) {
    const int i = f / a.m, j = f - i * a.m;
    double d = 0.0;
    for (int l = 0; l <= j; ++l) d += a.Ls[j * a.m + l] * N_lds[i * a.m + l];
    d = ok ? d * inv_eta : 0.0;
    a.dbg[2 + f] = d;
    a.U64[f] += d;
  }
  if (threadIdx.x == 0) {
    a.dbg[0] = rho;
    a.dbg[1] = ok ? eta : 0.0;
    if (!ok) a.flags[0] += 1;
    if (status_out) *status_out = ok ? 0.0 : -5.0;
    a.iter[0] += 1;
  }
  if (a.emit) {
    __syncthreads();
    double nxt[kMaxTM / kFinBlock];
    int n = 0;
    for (int f = threadIdx.x; f < TM; f += kFinBlock) {
      if (f < a.m) u0_out[f] = a.U64[f];
      nxt[n++] = (f + a.m < TM) ? a.U64[f + a.m] : a.u_init[f - (TM - a.m)];
    }
    __syncthreads();
    n = 0;
    for (int f = threadIdx.x; f < TM; f += kFinBlock) a.U64[f] = nxt[n++];
    __syncthreads();
  }
  for (int f = threadIdx.x; f < TM; f += kFinBlock) a.U32[f] = (float)a.U64[f];
}

static __global__ __launch_bounds__(kFinBlock) void finalize_kernel(const FinalizeArgs a) {
  finalize_body(a, a.u0_out, nullptr);
}

// --------------------------------------------------------------------- plant (FP64)
// x holds n <= Sys::N doubles; components beyond n are treated as zero and not written.
template <class Sys>
__global__ void plant_kernel(double *x, const double *u, double dt, int n, const typename Sys::Params p) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double xl[Sys::N], ul[Sys::M], xd[Sys::N];
  for (int r = 0; r < Sys::N; ++r) xl[r] = r < n ? x[r] : 0.0;
  for (int j = 0; j < Sys::M; ++j) ul[j] = u[j];
  Sys::xdot(p, xl, ul, xd);
  for (int r = 0; r < n; ++r) x[r] = xl[r] + dt * xd[r];
}

// ---------------------------------------------------------------------- diagnostics
static __global__ void normals_kernel(float *out, uint64_t it, uint32_t key0, uint32_t key1, int k0, int nk, int TM) {
  const int G = (TM + 3) / 4;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nk * G) return;
  const int kk = idx / G, g = idx - kk * G;
  float e[4];
  normals4((uint32_t)g, (uint32_t)(k0 + kk), it, key0, key1, e);
  for (int c = 0; c < 4; ++c) {
    const int f = g * 4 + c;
    if (f < TM) out[(size_t)kk * TM + f] = e[c];
  }
}

static __global__ void philox_kernel(const uint4 *ctr, uint4 *out, int n, uint32_t key0, uint32_t key1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = philox4x32_10(ctr[i], key0, key1);
}

}  // namespace mppi
