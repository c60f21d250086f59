// The MPPI iteration as three kernels (paper: Algorithm 1 with the likelihood-ratio
// running cost and update law of Section III-C), or two (below):
//
//   rollout<Sys>  the step-split body (4, 16 or 32 lanes sharing a sample's horizon) for
//                 systems whose cost does not act on the state, or the four-lane body
//                 (a DPP quad per sample; one lane with the LPS = 1 build) for the
//                 quadrotor, whose cost is split over the quad: draw the
//                 perturbations from Philox in registers, Euler-step the dynamics over
//                 the horizon, accumulate the path cost
//                 S_k = sum_i [q(x_{i+1}) + du'Mq du + u'R du + u'R u/2] + phi, where
//                 Mq = (R - A^-1 R A^-1)/2 and du ~ N(0, A Sigma A) (A = sqrt(nu) I or diagonal)
//                 (FP32 arithmetic per step, FP64 running sum), write S_k and the block
//                 minimum.
//   update        2-D grid over (sample chunk, noise group): rho = min_k S_k,
//                 w_k = exp(-(S_k - rho)/lambda) in FP64, regenerate the same normals and
//                 accumulate sum_k w_k eps_k in FP64; fixed-order reductions, no atomics.
//   finalize      one block: eta = sum_k w_k, dU = A L (sum_k w_k eps_k) / eta,
//                 U += dU (FP64 master, FP32 copy for the next rollout); on the last
//                 iteration of a control step emit u0 and apply the warm shift.
//
// The iteration also runs as two kernels (kFused): each rollout block keeps the normals it
// drew in LDS, weights its own samples against its own minimum rho_b and writes
// (rho_b, eta_b, N_b = sum_k exp(-(S_k - rho_b)/lambda) eps_k); the finalize rescales every
// block's partials by exp(-(rho_b - rho)/lambda), which turns them into the weights of the
// global minimum exactly (the sample-independent factor of the weights cancels in the
// normalised update, Section III-B).  Under cost-to-go weighting (step-split body) the same
// holds step by step, with the blocks' per-step minima and normalisers.
//
// The fused iteration's finalize runs as one block per four sequence components (the
// multi-block finalize): it reads the old sequence from a shadow that an extra rollout block
// copies, so its blocks can write the shifted sequence back without racing each other's
// reads.
#pragma once
#include "mppi_systems.h"

namespace mppi {

constexpr int kUpdGroups = 4;                        // noise groups per update block
constexpr int kUpdStrips = kBlock / kUpdGroups;      // sample strips per update block
static_assert(kUpdStrips % 16 == 0 && kUpdGroups * 4 * 16 <= kBlock, "update reduction layout");
constexpr int kUpdChunkMax = 2 * kBlock;             // samples per update block: 128, 256 or 512 (IterArgs)

struct IterArgs {
  const double *x0;        // [n]
  const double *U64;       // [T*m] FP64 master
  double *Ushadow;         // [T*m] fused: the master as the multi-block finalize reads it
                           // (copied by the extra rollout block, index n_roll_blocks), else NULL
  const float *U32;        // [T*m] FP32 copy of the nominal sequence
  double *S;               // [K] path costs
  double *blk_min;         // [n_roll_blocks]
  const uint64_t *iter;    // iteration counter (keys the noise)
  double *part;            // [n_kc][G*4] partial sums of w*eps
  double *eta_part;        // [n_kc] ([n_kc][T] with cost-to-go weights)
  double *pre;             // cost-to-go weights only: [T][K] sum of the first i step costs, else NULL
  double *rho_step;        // cost-to-go weights only: [T] min_k of the cost from step i onward
  double *blk_tail;        // cost-to-go, step-split body: [T][n_roll_blocks] each rollout block's
                           // min of the cost from step i onward (the update reduces them); else NULL
  uint32_t key0, key1;
  int n;                   // state dimension actually present in x0 (<= Sys::N)
  int K, T, m, G;          // G = ceil(T*m/4) noise groups per sample
  int n_roll_blocks, n_kc;
  float dt;
  float Mq[16];            // 1/2 (R - A^-1 R A^-1): quadratic likelihood-ratio term, m x m
  float Ls[16];            // A chol(Sigma), row-major m x m (lower)
  float R[16];             // m x m
  double inv_lambda;
  double *rho_out;         // update: this iteration's minimum path cost (written by one block)
  int upd_chunk;           // samples per update block (128, 256, or 512 with path weighting)
  double *plant_basis;     // multi-block finalize, last iteration of a plant step: the extra
  const double *plant_x;   // rollout block writes the plant basis of plant_x here
                           // ([Sys::M + 1][Sys::N]), else NULL
};

// Limits of the multi-block finalize and the fused variant: partial sums one finalize block
// merges (one per thread), sequence components per finalize block, LDS for a fused step-split
// rollout block's normals (several blocks share a CU), and the LDS a block may take (all of
// a gfx950 CU's: the four-lane body runs one block per CU).
constexpr int kMaxMergedParts = 1024;
constexpr int kFinOut = 4;
constexpr int kFinMultiBlock = 256;                  // threads of a multi-block finalize block
constexpr int kMaxFusedNormalsBytes = 32 * 1024;
constexpr int kMaxBlockLdsBytes = 160 * 1024;
constexpr int kQuadFusedAutoBlocks = 256;           // the MI355X's CUs

struct FinalizeArgs {
  double *U64;             // [T*m] FP64 master
  float *U32;              // [T*m]
  const double *rho;       // the iteration's minimum path cost (written by the update)
  const double *part;
  const double *eta_part;
  uint64_t *iter;
  int *flags;              // bit 0: an iteration had no finite cost
  double *dbg;             // [2 + T*m]: rho, eta, dU
  double *u0_out;          // [m]; written when emit != 0
  int T, m, G, n_kc;
  int emit;                // last iteration of the control step: emit u0 and shift
  int ctg;                 // cost-to-go weights: eta_part is [n_kc][T], one normaliser per step
  int multi;               // multi-block finalize (fused): ceil(T*m / kFinOut) blocks merge
  int n_parts;             //   the partials of n_parts rollout blocks
  const double *blk_min;   // multi-block: [n_parts] the rollout blocks' minima
  const double *Ushadow;   // multi-block: the master before this iteration
  const double *blk_tail;  // multi-block, cost-to-go: [T][n_parts] the rollout blocks' per-step minima
  double *rho_step;        // multi-block, cost-to-go: [T] receives each step's minimum
  double inv_lambda;
  double Ls[16];           // A chol(Sigma)
  double u_init[4];
};

// --------------------------------------------------------------------- plant (FP64)
// The harness plant step x <- x + dt xdot(x, u), FP64.  Every system is affine in its
// control, so xdot(x, u) = f0 + sum_j u_j (f_{j+1} - f0) with f0 = xdot(x, 0) and
// f_{j+1} = xdot(x, e_j): M + 1 lanes evaluate these in parallel, before u is known (in
// the finalize kernel, while the other waves wait on their loads), and one lane combines.
// Both plant kernels use the same two functions, so they agree bit for bit.  x holds
// n <= Sys::N doubles; components beyond n are treated as zero and not written.
template <class Sys>
__device__ __forceinline__ void plant_basis(const typename Sys::Params &p, const double *x, int n, int j,
                                            double *out) {
  double xl[Sys::N], ul[Sys::M];
  for (int r = 0; r < Sys::N; ++r) xl[r] = r < n ? x[r] : 0.0;
  for (int c = 0; c < Sys::M; ++c) ul[c] = c + 1 == j ? 1.0 : 0.0;
  Sys::xdot(p, xl, ul, out);
}
template <class Sys>
__device__ __forceinline__ void plant_combine(double *x, int n, double dt, const double (*basis)[Sys::N],
                                              const double *u) {
  for (int r = 0; r < n; ++r) {
    double d = basis[0][r];
    for (int c = 0; c < Sys::M; ++c) d = fma(u[c], basis[c + 1][r] - basis[0][r], d);
    x[r] = fma(dt, d, x[r]);
  }
}

// ------------------------------------------------------------------------ rollout
// One block of one controller (`blk` indexes the controller's blocks): 256 / LPS samples,
// LPS adjacent lanes per sample.  With LPS = 4 the four lanes of a DPP quad share a
// sample: lane j generates every fourth noise group (g = 4r + j) and broadcasts it (with
// the folded step, its fold) across the quad, a system with a decomposable cost splits it
// over the quad (each lane summing its share in FP64, the shares added after the horizon;
// per step with two DPP steps where the running total is recorded), and the dynamics run
// redundantly, so all four lanes hold the same state.  The single-controller kernel and the batched serving kernel both
// call this body, so a controller's results do not depend on what else shares a launch.
__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad_perm(1,0,3,2)
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad_perm(2,3,0,1)
  return v;
}
// Sum over a sample's LPS lanes; lane 0 of the group holds the fixed-order total.
template <int LPS>
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_f64<0xB1>(v);                            // quad_perm(1,0,3,2)
  v += dpp_f64<0x4E>(v);                            // quad_perm(2,3,0,1)
  if constexpr (LPS >= 16) {
    v += dpp_f64<0x124>(v);                         // row_ror:4
    v += dpp_f64<0x128>(v);                         // row_ror:8
  }
  if constexpr (LPS == 32) {                        // lane 0 adds lane 16's row total
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), (16 << 10) | 0x1F);   // lane ^ 16
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), (16 << 10) | 0x1F);
    v += __hiloint2double(hi, lo);
  }
  return v;
}
__device__ __forceinline__ float quad_max(float v) {
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false)));
  return v;
}

// Rollout variants (compile-time, so the default path carries none of their code):
// kRecordPrefix records each sample's cost before every step (cost-to-go weighting);
// kCrash applies the system's crash indicator (systems with Sys::kCrash only);
// kStepSplit selects the step-split body below (systems with Sys::kStepSplit; with
// kRecordPrefix or alone).
// kDiagLR: Ls and Mq are diagonal, so the noise and likelihood-ratio products keep their
// diagonal terms only -- the general FMA chains add exact zeros to them, so both forms give
// the same values bit for bit.
// kFused (path weighting): the rollout block also writes its weighted partial sums, so no
// update kernel runs and the finalize merges the blocks' partials.
enum { kRecordPrefix = 1, kCrashOn = 2, kStepSplit = 4, kDiagLR = 8, kFused = 16 };
// Inside the four-lane body only (never a launch variant): the system's split cost reads
// all its data from registers, so its LDS pass is left out.
constexpr int kRegOnly = 32;

// Systems with their own folded FP32 Euler step for the rollout (Sys::euler_folded, with
// Sys::init_state and Sys::fold_controls), and systems whose state cost has a per-step
// constant that the per-step control cost carries (Sys::step_const).
template <class Sys, class = void>
struct has_folded_euler : std::false_type {};
template <class Sys>
struct has_folded_euler<Sys, std::void_t<decltype(Sys::kFoldedEuler)>> : std::bool_constant<Sys::kFoldedEuler> {};
template <class Sys, class = void>
struct has_step_const : std::false_type {};
template <class Sys>
struct has_step_const<Sys, std::void_t<decltype(Sys::kStepConst)>> : std::bool_constant<Sys::kStepConst> {};
// The folded step runs in every variant of such a system (under the crash indicator only
// while the sample has not crashed).
template <class Sys, int Mode>
constexpr bool folded_step() { return has_folded_euler<Sys>::value; }

// The likelihood-ratio control terms of one step (m = 4) from its four normals e:
// du = A L e, then du'Mq du + (R u_i)'du + u_i'R u_i / 2 as sum_r du_r ((Mq du)_r + (R u_i)_r)
// + C_i, with ru = R u_i and c = C_i.  The diagonal form keeps the diagonal products only
// (the general chains add exact zeros to them: the same bits).
template <int Mode>
__device__ __forceinline__ float lr_terms4(const IterArgs &a, const float *e, float4 ru, float c) {
  constexpr int M = 4;
  const float rv[4] = {ru.x, ru.y, ru.z, ru.w};
  float du[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    if constexpr ((Mode & kDiagLR) != 0) {
      du[r] = fmaf(a.Ls[r * M + r], e[r], 0.f);
    } else {
      float t = 0.f;
#pragma unroll
      for (int l = 0; l <= r; ++l) t = fmaf(a.Ls[r * M + l], e[l], t);
      du[r] = t;
    }
  }
  float acc = c;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    float t = rv[r];
    if constexpr ((Mode & kDiagLR) != 0) {
      t = fmaf(a.Mq[r * M + r], du[r], t);
    } else {
#pragma unroll
      for (int j = 0; j < M; ++j) t = fmaf(a.Mq[r * M + j], du[j], t);
    }
    acc = fmaf(du[r], t, acc);
  }
  return acc;
}

// Whether the four-lane body sums a sample's path cost per lane (each lane its share of every
// step, in FP64; the lanes' sums added in a fixed tree at the end) rather than per step across
// the quad: wherever no step's running total is recorded.
template <class Sys, int LPS, int Mode>
constexpr bool lane_sums() { return LPS == 4 && Sys::kSplitCost && (Mode & kRecordPrefix) == 0; }

// One horizon step of one sample from the four normals `e` of its noise group.  With the
// folded step, sU holds the fold of each step's nominal controls and nf is the fold of the
// step's perturbation (e is then used only by the one-lane likelihood-ratio terms).  With
// the four-lane split cost (m = 4), lr_base is this lane's share of the step's
// likelihood-ratio terms (all of them in the lane that drew the step's group, zero in the
// others).  With lane_sums, S is this lane's share of the path cost.
template <class Sys, int LPS, int Mode>
__device__ __forceinline__ void rollout_step(const IterArgs &a, const typename Sys::Params &p, const StageView &sv,
                                             const typename Sys::Regs &rg, float lr_base, const float *sU,
                                             const float *sRU, const float *sC, int i, int s, int lane_j, int k,
                                             const float e[4], float4 nf, float *x, double &S, bool &crashed) {
  if constexpr ((Mode & kRecordPrefix) != 0)
    if (lane_j == 0 && k < a.K) a.pre[(size_t)i * a.K + k] = S;        // cost of steps before i
  constexpr int N = Sys::N, M = Sys::M;
  float du[M], v[M], xd[N];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    float t = 0.f;
    if constexpr ((Mode & kDiagLR) != 0) {
      t = fmaf(a.Ls[j * M + j], e[s * M + j], 0.f);
    } else {
#pragma unroll
      for (int l = 0; l <= j; ++l) t += a.Ls[j * M + l] * e[s * M + l];
    }
    du[j] = t;
    v[j] = sU[i * M + j] + t;
  }
  if constexpr (folded_step<Sys, Mode>()) {
    static_assert(M == 4, "the folded step maps four normals");
    // a crashed rollout stays where it is (its quad agrees, so the branch is quad-uniform)
    if ((Mode & kCrashOn) == 0 || !crashed) Sys::euler_folded(p, a.dt, x, reinterpret_cast<const float4 *>(sU)[i], nf);
  } else if constexpr ((Mode & kCrashOn) != 0) {
    Sys::xdot(p, x, v, xd);
    if (!crashed) {                                 // a crashed rollout stays where it is
#pragma unroll
      for (int r = 0; r < N; ++r) x[r] += a.dt * xd[r];
    }
  } else {
    Sys::xdot(p, x, v, xd);
#pragma unroll
    for (int r = 0; r < N; ++r) x[r] += a.dt * xd[r];
  }
  // likelihood-ratio control terms du'Mq du + (R u_i)'du + u_i'R u_i / 2: with a split
  // cost (m = 4) the lane that drew the step's group formed them (lr_terms4) and they join
  // the state cost in the same quad sum
  constexpr bool kSplitLR = LPS == 4 && Sys::kSplitCost && M == 4;
  float quad = 0.f, lin = 0.f, lr_in = 0.f;         // lr_in: this lane's share (split form)
  if constexpr (kSplitLR) {
    lr_in = lr_base;
  } else {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      float t = 0.f;
      if constexpr ((Mode & kDiagLR) != 0) {
        t = fmaf(a.Mq[r * M + r], du[r], 0.f);
      } else {
#pragma unroll
        for (int j = 0; j < M; ++j) t += a.Mq[r * M + j] * du[j];
      }
      quad += du[r] * t;
      lin += sRU[i * M + r] * du[r];
    }
  }
  constexpr bool kLane = lane_sums<Sys, LPS, Mode>();
  float q;
  if constexpr ((Mode & kCrashOn) != 0) {          // crash indicator: sticky, crash cost per step
    static_assert(Sys::kCrash, "system has no crash indicator");
    float hit;
    if constexpr (LPS == 4) {
      q = Sys::template q_part_crash<(Mode & kRegOnly) != 0>(p, sv, rg, x, lane_j, 4, lr_in, hit);
      if constexpr (!kLane) q = quad_sum(q);
      hit = quad_max(hit);
    } else {
      q = Sys::template q_part_crash<false>(p, sv, rg, x, 0, 1, 0.f, hit);
    }
    crashed = crashed || hit > 0.f;
    if (crashed && (!kLane || lane_j == 0)) q += p.crash;
  } else if constexpr (LPS == 4 && Sys::kSplitCost) {
    q = Sys::template q_part<(Mode & kRegOnly) != 0>(p, sv, rg, x, lane_j, 4, lr_in);
    if constexpr (!kLane) q = quad_sum(q);
  } else {
    q = Sys::q(p, sv, x);
  }
  const float qt = kSplitLR ? q : q + (quad + lin + sC[i]);
  S += (double)qt;
}

// The fused iteration's block tail: the block's weights against its own minimum bm, then its
// partial sums sum_k w_k eps_k over its samples in sample order and its normaliser.  sE holds
// the block's normals [SPB][G*4] (published by block_min's barriers), sW [SPB] doubles;
// `owner` marks the lane that holds sample sb's path cost S (`valid`: a sample of this
// controller).
template <int SPB>
__device__ __forceinline__ void fused_tail(const IterArgs &a, int blk, int M, bool owner, int sb, bool valid, double S,
                                           double bm, const float *sE, double *sW) {
  if (owner) sW[sb] = valid && S < __builtin_inf() ? exp(-(S - bm) * a.inv_lambda) : 0.0;
  __syncthreads();
  // a thread per four components (four independent FMA chains, one 16-byte read per sample;
  // F is a multiple of four, so a quad never leaves its sample's row), each summed over the
  // samples in order
  const int TM = a.T * M, F = a.G * 4, nq = (TM + 3) / 4;
  for (int q = threadIdx.x; q < nq; q += kBlock) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
    for (int j = 0; j < SPB; ++j) {
      const float4 e = *reinterpret_cast<const float4 *>(sE + j * F + 4 * q);
      const double w = sW[j];
      acc[0] = fma(w, (double)e.x, acc[0]);
      acc[1] = fma(w, (double)e.y, acc[1]);
      acc[2] = fma(w, (double)e.z, acc[2]);
      acc[3] = fma(w, (double)e.w, acc[3]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (4 * q + c < TM) a.part[(size_t)blk * F + 4 * q + c] = acc[c];
  }
  if (threadIdx.x == kBlock - 1) {                  // the last wave has the fewest quads
    double e = 0.0;
#pragma unroll
    for (int j = 0; j < SPB; ++j) e += sW[j];
    a.eta_part[blk] = e;
  }
}

template <class Sys, int LPS, int Mode>
__device__ __forceinline__ void rollout_body(const IterArgs &a, const typename Sys::Params &p, const double *x0,
                                             int blk, float4 *lds4) {
  constexpr int N = Sys::N, M = Sys::M;
  constexpr int SPG = 4 / M;                        // steps per noise group
  float *sU = reinterpret_cast<float *>(lds4);      // [T*M]
  float *sRU = sU + a.T * M;                        // [T*M]  R u_i
  float *sC = sRU + a.T * M;                        // [T]    u_i'R u_i / 2
  float *sSys = sU + ((2 * a.T * M + ((a.T + 3) & ~3) + 3) & ~3);   // system staging, 16-B aligned
  // kFused: the block's normals [SPB][G*4] and its samples' weights [SPB] (FP64), after the
  // system's staging (16-B aligned)
  constexpr int SPB = kBlock / LPS;
  static_assert((Mode & kFused) == 0 || (Mode & kRecordPrefix) == 0, "fused: path weighting only");
  float *sE = nullptr;
  double *sW = nullptr;
  if constexpr ((Mode & kFused) != 0) {
    sE = sSys + ((Sys::staged_floats(p) + 3) & ~3);
    sW = reinterpret_cast<double *>(sE + SPB * a.G * 4);
  }
  __shared__ double red[4];

  const uint64_t it = *a.iter;
  constexpr bool kFold = folded_step<Sys, Mode>();
  // Preamble loads first (start state, this thread's first control, then the system's
  // staging loads), so their memory latencies overlap instead of following each other.
  float x[N];
  if constexpr (kFold) {
    Sys::init_state(x0, a.n, x);
  } else {
#pragma unroll
    for (int r = 0; r < N; ++r) x[r] = r < a.n ? (float)x0[r] : 0.f;
  }
  float u_first[M];
#pragma unroll
  for (int j = 0; j < M; ++j) u_first[j] = threadIdx.x < a.T ? a.U32[threadIdx.x * M + j] : 0.f;
  int ti = 0, tj = 0;                               // every thread computes the same origin
  Sys::stage(p, sSys, x0, &ti, &tj);
  for (int i = threadIdx.x; i < a.T; i += kBlock) {
    float u[M];
#pragma unroll
    for (int j = 0; j < M; ++j) u[j] = i == threadIdx.x ? u_first[j] : a.U32[i * M + j];
    float c = 0.f;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      float s = 0.f;
#pragma unroll
      for (int j = 0; j < M; ++j) s += a.R[r * M + j] * u[j];
      if constexpr (!kFold) sU[i * M + r] = u[r];
      sRU[i * M + r] = s;
      c += u[r] * s;
    }
    if constexpr (kFold) reinterpret_cast<float4 *>(sU)[i] = Sys::fold_controls(p, u[0], u[1], u[2], u[3]);
    if constexpr (has_step_const<Sys>::value) sC[i] = fmaf(0.5f, c, Sys::step_const(p));
    else sC[i] = 0.5f * c;
  }
  __syncthreads();
  const StageView sv{sSys, ti, tj};
  // the folded step's map of the normals: W[l] = the fold of column l of A chol(Sigma)
  float4 W[4];
  if constexpr (kFold) {
#pragma unroll
    for (int l = 0; l < 4; ++l) W[l] = Sys::fold_controls(p, a.Ls[l], a.Ls[4 + l], a.Ls[8 + l], a.Ls[12 + l]);
  }

  const int lane_j = threadIdx.x % LPS;
  typename Sys::Regs rg;                            // per-lane register copy of system data
  Sys::load_regs(p, sv, lane_j, LPS, rg);
  const int k = blk * (kBlock / LPS) + threadIdx.x / LPS;
  double S = 0.0;
  bool crashed = false;                             // set only in the kCrashOn variant
  if constexpr (LPS == 1) {
    for (int g = 0; g < a.G; ++g) {
      float e[4];
      normals4((uint32_t)g, (uint32_t)k, it, a.key0, a.key1, e);
#pragma unroll
      for (int s = 0; s < SPG; ++s) {
        const int i = g * SPG + s;
        if (i < a.T) {
          float4 nf = make_float4(0.f, 0.f, 0.f, 0.f);
          if constexpr (kFold) nf = Sys::template fold_noise<(Mode & kDiagLR) != 0>(W, e + s * M);
          rollout_step<Sys, LPS, Mode>(a, p, sv, rg, 0.f, sU, sRU, sC, i, s, 0, k, e, nf, x, S, crashed);
        }
      }
    }
  } else {
    static_assert(LPS == 4, "LPS is 1 or 4");
    // One chunk of four noise groups: lane j draws group g0 + j and the quad takes the groups
    // in turn.  kFull: all four groups lie inside the horizon (no group is guarded, nor, with
    // one step per group, any step).  MD carries kRegOnly when the system's cost needs no
    // LDS pass (decided once per block, so the step loop holds no such branch).
    auto chunk = [&](int g0, auto full_c, auto mode_c) {
      constexpr bool kFull = decltype(full_c)::value;
      constexpr int MD = decltype(mode_c)::value;
      float mine[4];
      normals4((uint32_t)(g0 + lane_j), (uint32_t)k, it, a.key0, a.key1, mine);
      if constexpr ((MD & kFused) != 0)             // kept for the block's partial sums
        if (kFull || g0 + lane_j < a.G)
          *reinterpret_cast<float4 *>(sE + ((threadIdx.x / LPS) * a.G + g0 + lane_j) * 4) =
              make_float4(mine[0], mine[1], mine[2], mine[3]);
      // split cost (m = 4, one step per group): this lane's step's likelihood-ratio terms,
      // once per chunk (a lane past the horizon forms those of the last step, never used)
      float lr_mine = 0.f;
      if constexpr (LPS == 4 && Sys::kSplitCost && M == 4) {
        const int im = min(g0 + lane_j, a.T - 1);
        lr_mine = lr_terms4<MD>(a, mine, reinterpret_cast<const float4 *>(sRU)[im], sC[im]);
      }
      // folded step (m = 4, one step per group): the lane that drew a group folds its
      // perturbation once and the quad broadcasts the fold instead of the normals
      float4 nf_mine = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (kFold) nf_mine = Sys::template fold_noise<(MD & kDiagLR) != 0>(W, mine);
#define MPPI_QUAD_GROUP(J)                                                              \
      if (kFull || g0 + J < a.G) {                                                      \
        float e[4] = {0.f, 0.f, 0.f, 0.f};          /* the normals, if not folded */    \
        float4 nf = make_float4(0.f, 0.f, 0.f, 0.f);                                    \
        if constexpr (kFold) {                                                          \
          nf = make_float4(quad_bcast<J>(nf_mine.x), quad_bcast<J>(nf_mine.y), quad_bcast<J>(nf_mine.z), \
                           quad_bcast<J>(nf_mine.w));                                   \
        } else {                                                                        \
          for (int c = 0; c < 4; ++c) e[c] = quad_bcast<J>(mine[c]);                    \
        }                                                                               \
        _Pragma("unroll") for (int s = 0; s < SPG; ++s) {                               \
          const int i = (g0 + J) * SPG + s;                                             \
          if ((kFull && SPG == 1) || i < a.T)                                           \
            rollout_step<Sys, LPS, MD>(a, p, sv, rg, lane_j == J ? lr_mine : 0.f, sU, sRU, sC, i, s, lane_j, k, e, nf, \
                                       x, S, crashed);                                 \
        }                                                                               \
      }
      MPPI_QUAD_GROUP(0)
      MPPI_QUAD_GROUP(1)
      MPPI_QUAD_GROUP(2)
      MPPI_QUAD_GROUP(3)
#undef MPPI_QUAD_GROUP
    };
    auto run = [&](auto mode_c) {
      int g0 = 0;
      for (; g0 + 4 <= a.G; g0 += 4) chunk(g0, std::true_type{}, mode_c);
      if (g0 < a.G) chunk(g0, std::false_type{}, mode_c);
    };
    if (Sys::lds_pass(p, LPS)) run(std::integral_constant<int, Mode>{});
    else run(std::integral_constant<int, Mode | kRegOnly>{});
  }
  if constexpr (lane_sums<Sys, LPS, Mode>()) S = group_sum<LPS>(S);   // the lanes' shares, fixed order
  S += (double)Sys::phi(p, x);
  if (!isfinite(S)) S = __builtin_inf();
  const bool valid = k < a.K && lane_j == 0;
  if (valid) a.S[k] = S;
  const double bm = block_min(valid ? S : __builtin_inf(), red);
  if (threadIdx.x == 0) a.blk_min[blk] = bm;
  if constexpr ((Mode & kFused) != 0) fused_tail<SPB>(a, blk, M, lane_j == 0, threadIdx.x / LPS, valid, S, bm, sE, sW);
}

// ------------------------------------------------------------- step-split rollout
// For a system whose cost does not act back on its state (path weighting, no crash
// indicator) the LPS lanes of a sample (4 or 16) share its horizon by noise group.  Per
// chunk of LPS groups, lane j draws group g0 + j and forms the perturbations of that
// group's steps and their likelihood-ratio terms; then every lane steps the dynamics
// through the whole chunk, taking group g0 + jj's perturbations from lane jj by a DPP
// broadcast, and lane j keeps the (cost-relevant) state after each of its own steps;
// after the chunk lane j evaluates the state cost at those states.  So the noise and the
// cost are computed once per step (not once per lane), and only the short dynamics
// chain is redundant.  The per-step cost is the FP32 expression of the four-lane body;
// each lane sums its steps in FP64 and the lanes' sums are added in a fixed tree.  Under
// cost-to-go weighting (kRecordPrefix) the running cost before every step is recorded
// by the lane owning the step, from an FP64 scan of the lanes' step costs across the
// group; the path cost is the same tree sum in both variants, so the two weightings see
// bitwise the same S.

template <class Sys, int LPS, int Mode>
__device__ __forceinline__ void rollout_body_split(const IterArgs &a, const typename Sys::Params &p,
                                                   const double *x0, int blk, float4 *lds4) {
  static_assert((Mode & kCrashOn) == 0, "the step-split body has no crash indicator");
  static_assert(Sys::kStepSplit, "system cost acts on the state");
  constexpr int N = Sys::N, M = Sys::M, NQ = Sys::NQ;
  constexpr bool kFusedCtg = (Mode & kFused) != 0 && (Mode & kRecordPrefix) != 0;
  constexpr int SPG = 4 / M;                        // steps per noise group
  constexpr int SPB = kBlock / LPS;                 // samples per block
  float *sU = reinterpret_cast<float *>(lds4);      // [T*M]
  float *sRU = sU + a.T * M;                        // [T*M]  R u_i
  float *sC = sRU + a.T * M;                        // [T]    u_i'R u_i / 2
  // kFused: the block's normals [SPB][G*4] and its samples' weights [SPB] (FP64); cost-to-go
  // with blk_tail: the running cost before each step [SPB][T] and the path costs [SPB] (FP64);
  // both (the fused cost-to-go iteration): the normals, then the running costs (which become
  // the samples' per-step weights), the path costs and the block's per-step minima [T]
  float *sE = sU + ((2 * a.T * M + ((a.T + 3) & ~3) + 3) & ~3);
  double *sW = reinterpret_cast<double *>(sE + SPB * a.G * 4);
  double *sPre = kFusedCtg ? sW : reinterpret_cast<double *>(sE);
  __shared__ double red[4];

  const uint64_t it = *a.iter;
  float x[N];
#pragma unroll
  for (int r = 0; r < N; ++r) x[r] = r < a.n ? (float)x0[r] : 0.f;
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
  __syncthreads();

  const int lane_j = threadIdx.x % LPS;
  const int k = blk * (kBlock / LPS) + threadIdx.x / LPS;
  double Sp = 0.0;                                  // this lane's steps
  double P = 0.0;                                   // running cost (kRecordPrefix only)
  for (int g0 = 0; g0 < a.G; g0 += LPS) {
    // this lane's group: perturbations du = A L eps and likelihood-ratio terms of its steps
    const int g = g0 + lane_j;
    float e[4];
    normals4((uint32_t)g, (uint32_t)k, it, a.key0, a.key1, e);
    if constexpr ((Mode & kFused) != 0)
      if (g < a.G)
        *reinterpret_cast<float4 *>(sE + ((threadIdx.x / LPS) * a.G + g) * 4) = make_float4(e[0], e[1], e[2], e[3]);
    float du[4], lr[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      const int ic = min(g * SPG + s, a.T - 1);    // steps past the horizon are never used
#pragma unroll
      for (int j = 0; j < M; ++j) {
        float t = 0.f;
        if constexpr ((Mode & kDiagLR) != 0) {
          t = fmaf(a.Ls[j * M + j], e[s * M + j], 0.f);
        } else {
#pragma unroll
          for (int l = 0; l <= j; ++l) t += a.Ls[j * M + l] * e[s * M + l];
        }
        du[s * M + j] = t;
      }
      float quad = 0.f, lin = 0.f;
#pragma unroll
      for (int r = 0; r < M; ++r) {
        float t = 0.f;
        if constexpr ((Mode & kDiagLR) != 0) {
          t = fmaf(a.Mq[r * M + r], du[s * M + r], 0.f);
        } else {
#pragma unroll
          for (int j = 0; j < M; ++j) t += a.Mq[r * M + j] * du[s * M + j];
        }
        quad += du[s * M + r] * t;
        lin += sRU[ic * M + r] * du[s * M + r];
      }
      lr[s] = quad + lin + sC[ic];
    }
    // every lane: the dynamics through the chunk; lane jj keeps the states after group jj's steps
    float xq[SPG][NQ];
#pragma unroll
    for (int s = 0; s < SPG; ++s)
#pragma unroll
      for (int c = 0; c < NQ; ++c) xq[s][c] = 0.f;
    // a full chunk runs without horizon checks (one basic block, so the control loads
    // are scheduled ahead of the steps that use them); only the last chunk checks
    auto chunk = [&](auto checked) {
      constexpr bool kChecked = decltype(checked)::value;
      if constexpr (Sys::kOwnChunk) {
        Sys::template chunk<LPS, SPG, kChecked>(p, a.T, a.dt, sU, du, g0, lane_j, x, xq);
      } else {
        StaticFor<0, LPS>::run([&](auto jc) {
          constexpr int JJ = decltype(jc)::value;
          const int i0 = (g0 + JJ) * SPG;
          if (!kChecked || i0 < a.T) {
            float db[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) db[c] = group_bcast<LPS, JJ>(du[c]);
            const bool mine = lane_j == JJ;
#pragma unroll
            for (int s = 0; s < SPG; ++s) {
              const int i = i0 + s;
              if (!kChecked || i < a.T) {
                float v[M], xd[N], t[NQ];
#pragma unroll
                for (int j = 0; j < M; ++j) v[j] = sU[i * M + j] + db[s * M + j];
                Sys::xdot(p, x, v, xd);
#pragma unroll
                for (int r = 0; r < N; ++r) x[r] += a.dt * xd[r];
                Sys::cost_state(x, t);
#pragma unroll
                for (int c = 0; c < NQ; ++c) xq[s][c] = mine ? t[c] : xq[s][c];
              }
            }
          }
        });
      }
    };
    if ((g0 + LPS) * SPG <= a.T) chunk(std::false_type{});
    else chunk(std::true_type{});
    // this lane's steps: state cost + likelihood-ratio terms
    float qt[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      qt[s] = 0.f;
      if (g * SPG + s < a.T) {
        qt[s] = Sys::q_step(p, xq[s]) + lr[s];
        Sp += (double)qt[s];
      }
    }
    if constexpr ((Mode & kRecordPrefix) != 0) {
      // cost-to-go weighting: the running cost before each of this lane's steps (the
      // running total, the lanes before this one by an FP64 scan across the group, this
      // lane's earlier steps), written by the lane that owns the step
      double own = 0.0;
#pragma unroll
      for (int s = 0; s < SPG; ++s) own += (double)qt[s];   // 0 past the horizon
      const double incl = group_scan_incl_f64<LPS>(own, lane_j);
      double r = P + group_excl_of_incl_f64<LPS>(incl, lane_j);
#pragma unroll
      for (int s = 0; s < SPG; ++s) {
        const int i = g * SPG + s;
        if (!kFusedCtg && i < a.T && k < a.K) a.pre[(size_t)i * a.K + k] = r;   // the update reads these
        if (a.blk_tail && i < a.T) sPre[(threadIdx.x / LPS) * a.T + i] = r;
        r += (double)qt[s];
      }
      P += group_bcast_f64<LPS, LPS - 1>(incl);
    }
  }
  double S = group_sum<LPS>(Sp) + (double)Sys::phi(p, x);
  if (!isfinite(S)) S = __builtin_inf();
  const bool valid = k < a.K && lane_j == 0;
  if (valid) a.S[k] = S;
  const double bm = block_min(valid ? S : __builtin_inf(), red);
  if (threadIdx.x == 0) a.blk_min[blk] = bm;
  if constexpr ((Mode & kRecordPrefix) != 0) {
    // the block's minimum of each step's cost from that step onward, S - (cost before it), from
    // the running costs its lanes kept in LDS (published by block_min's barriers): the update
    // reduces these instead of a separate pass over the [T][K] prefix costs
    if (a.blk_tail) {
      double *sS = sPre + SPB * a.T;
      double *sRho = sS + SPB;                      // kFusedCtg: the block's per-step minima
      if (lane_j == 0) sS[threadIdx.x / LPS] = valid ? S : __builtin_inf();
      __syncthreads();
      for (int i = threadIdx.x; i < a.T; i += kBlock) {
        double m = __builtin_inf();
        for (int sb = 0; sb < SPB; ++sb) {
          const double sv = sS[sb];
          m = fmin(m, sv < __builtin_inf() ? sv - sPre[sb * a.T + i] : __builtin_inf());
        }
        a.blk_tail[(size_t)i * a.n_roll_blocks + blk] = m;
        if constexpr (kFusedCtg) sRho[i] = m;
      }
      if constexpr (kFusedCtg) {
        // the fused cost-to-go iteration: each sample's per-step weights against the block's
        // own per-step minima, w = exp(-((S - cost before step i) - rho_b,i) / lambda) (in
        // place of the running costs), then the block's per-step sums in sample order: for
        // component f of step i = f / m, sum_k w_k,i eps_k,f, and eta_b,i = sum_k w_k,i
        __syncthreads();
        for (int q = threadIdx.x; q < SPB * a.T; q += kBlock) {
          const int sb = q / a.T, i = q - sb * a.T;
          const double sv = sS[sb];
          sPre[q] = sv < __builtin_inf() ? exp(-((sv - sPre[q]) - sRho[i]) * a.inv_lambda) : 0.0;
        }
        __syncthreads();
        const int TM = a.T * M, F = a.G * 4;
        for (int f = threadIdx.x; f < TM; f += kBlock) {
          const int i = f / M;
          double acc = 0.0;
#pragma unroll
          for (int sb = 0; sb < SPB; ++sb) acc = fma(sPre[sb * a.T + i], (double)sE[sb * F + f], acc);
          a.part[(size_t)blk * F + f] = acc;
        }
        for (int i = threadIdx.x; i < a.T; i += kBlock) {
          double e = 0.0;
#pragma unroll
          for (int sb = 0; sb < SPB; ++sb) e += sPre[sb * a.T + i];
          a.eta_part[(size_t)blk * a.T + i] = e;
        }
      }
    }
  }
  if constexpr ((Mode & kFused) != 0 && !kFusedCtg)
    fused_tail<SPB>(a, blk, M, lane_j == 0, threadIdx.x / LPS, valid, S, bm, sE, sW);
}

// Multi-block finalize: the block past a controller's rollout blocks, off the critical paths:
// the master as this iteration's finalize reads it (its blocks write the shifted sequence into
// U64 while others still read the old one) and, before a plant step, the plant basis of the
// plant state (the finalize combines it with the emitted control).
template <class Sys>
__device__ __forceinline__ void shadow_block(const IterArgs &a, const typename Sys::Params &p) {
  for (int f = threadIdx.x; f < a.T * a.m; f += kBlock) a.Ushadow[f] = a.U64[f];
  if (a.plant_basis && (int)threadIdx.x <= Sys::M)
    plant_basis<Sys>(p, a.plant_x, a.n, threadIdx.x, a.plant_basis + threadIdx.x * Sys::N);
}

// The body a rollout variant runs (the single-controller and the batched kernels alike).
template <class Sys, int LPS, int Mode>
__device__ __forceinline__ void rollout_any(const IterArgs &a, const typename Sys::Params &p, const double *x0,
                                            int blk, float4 *lds4) {
  if constexpr ((Mode & kStepSplit) != 0) {
    rollout_body_split<Sys, LPS, Mode>(a, p, x0, blk, lds4);
  } else {
    rollout_body<Sys, LPS, Mode>(a, p, x0, blk, lds4);
  }
}

template <class Sys, int LPS, int Mode>
__global__ __launch_bounds__(kBlock) void rollout_kernel(const IterArgs a, const typename Sys::Params p) {
  extern __shared__ float4 lds4[];
  if (a.Ushadow && (int)blockIdx.x == a.n_roll_blocks) {
    shadow_block<Sys>(a, p);
    return;
  }
  rollout_any<Sys, LPS, Mode>(a, p, a.x0, blockIdx.x, lds4);
}

// Minimum over the rollout blocks' minima (every thread gets it).
__device__ __forceinline__ double global_min(const double *blk_min, int n, double *red) {
  double v = threadIdx.x < n ? blk_min[threadIdx.x] : __builtin_inf();
  for (int b = threadIdx.x + kBlock; b < n; b += kBlock) v = fmin(v, blk_min[b]);
  return block_min(v, red);
}

// ------------------------------------------------------------------------- update
// grid (n_kc, ceil(G / kUpdGroups)).  Thread t handles noise group gcb*kUpdGroups +
// t % kUpdGroups for the upd_chunk / kUpdStrips samples of strip t / kUpdGroups of this
// block's chunk of upd_chunk samples.
__device__ __forceinline__ void update_body(const IterArgs &a, int kc, int gcb) {
  __shared__ double w[kUpdChunkMax];
  __shared__ double acc_lds[kUpdStrips][kUpdGroups][4];
  __shared__ double red[4];
  const int chunk = a.upd_chunk, ppt = chunk / kUpdStrips;
  // the iteration counter before the minimum's barriers (a load after a barrier waits for it)
  const uint64_t it = *a.iter;
  // this thread's samples of the chunk (tid, tid + 256): costs in flight with the minima
  constexpr int kOwn = kUpdChunkMax / kBlock;
  double s_own[kOwn];
#pragma unroll
  for (int o = 0; o < kOwn; ++o) {
    const int kk = threadIdx.x + o * kBlock, k = kc * chunk + kk;
    s_own[o] = kk < chunk && k < a.K ? a.S[k] : __builtin_inf();
  }
  const double rho = global_min(a.blk_min, a.n_roll_blocks, red);
  if (kc == 0 && gcb == 0 && threadIdx.x == 0) *a.rho_out = rho;
  {
    double wsum = 0.0;                              // this thread's weights, in order
#pragma unroll
    for (int o = 0; o < kOwn; ++o) {
      const int kk = threadIdx.x + o * kBlock;
      double wk = 0.0;
      if (rho < __builtin_inf() && s_own[o] < __builtin_inf()) wk = exp(-(s_own[o] - rho) * a.inv_lambda);
      if (kk < chunk) w[kk] = wk;
      wsum += wk;
    }
    if (gcb == 0) {
      const double e = block_sum(wsum, red);
      if (threadIdx.x == 0) a.eta_part[kc] = e;
    }
  }
  __syncthreads();
  const int gl = threadIdx.x % kUpdGroups, strip = threadIdx.x / kUpdGroups;
  const int g = gcb * kUpdGroups + gl;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (g < a.G) {
    for (int r = 0; r < ppt; ++r) {
      const int kl = strip * ppt + r;
      const double wk = w[kl];
      if (wk != 0.0) {
        float e[4];
        normals4((uint32_t)g, (uint32_t)(kc * chunk + kl), it, a.key0, a.key1, e);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = fma(wk, (double)e[c], acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) acc_lds[strip][gl][c] = acc[c];
  __syncthreads();
  // fixed-order two-level sum over the strips: 16 runs of kUpdStrips/16, then the runs
  __shared__ double runs[16][kUpdGroups * 4];
  {
    const int slot = threadIdx.x % (kUpdGroups * 4), run = threadIdx.x / (kUpdGroups * 4);
    if (run < 16) {
      const int gg = slot / 4, c = slot % 4;
      double s = 0.0;
      for (int st = run * (kUpdStrips / 16); st < (run + 1) * (kUpdStrips / 16); ++st) s += acc_lds[st][gg][c];
      runs[run][slot] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < kUpdGroups * 4) {
    const int gg = threadIdx.x / 4, c = threadIdx.x % 4;
    const int gabs = gcb * kUpdGroups + gg;
    double s = 0.0;
    for (int r = 0; r < 16; ++r) s += runs[r][threadIdx.x];
    if (gabs < a.G) a.part[(size_t)kc * (a.G * 4) + gabs * 4 + c] = s;
  }
}

static __global__ __launch_bounds__(kBlock) void update_kernel(const IterArgs a) {
  update_body(a, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------ cost-to-go weighting (option)
// Step i of sample k is weighted by its cost from step i onward, S_k - pre[i][k] (the
// update law's S(tau_{i,k})): w = exp(-((S_k - pre[i][k]) - rho_i) / lambda), with rho_i
// and eta_i per step.
static __global__ __launch_bounds__(kBlock) void stepmin_kernel(const IterArgs a) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const double *pre_i = a.pre + (size_t)i * a.K;
  double v = __builtin_inf();
  // loads issued kB samples at a time, ahead of their use (one memory round trip per batch)
  constexpr int kB = 16;
  for (int k0 = threadIdx.x; k0 < a.K; k0 += kB * kBlock) {
    double sv[kB], pv[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int k = k0 + j * kBlock;
      sv[j] = k < a.K ? a.S[k] : __builtin_inf();
      pv[j] = k < a.K ? pre_i[k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kB; ++j) v = fmin(v, sv[j] < __builtin_inf() ? sv[j] - pv[j] : __builtin_inf());
  }
  v = block_min(v, red);
  if (threadIdx.x == 0) a.rho_step[i] = v;
}

static __global__ __launch_bounds__(kBlock) void update_ctg_kernel(const IterArgs a) {
  // The chunk has at most kBlock samples under cost-to-go weighting (one per thread), and
  // m is 1, 2 or 4, so the steps of this block's groups are exactly the steps whose first
  // component lies in them: their weights are computed once, for the normalisers, and
  // kept in LDS for the accumulation.
  constexpr int kMaxSteps = kUpdGroups * 4;
  __shared__ double acc_lds[kUpdStrips][kUpdGroups][4];
  __shared__ double runs[16][kUpdGroups * 4];
  __shared__ double w_lds[kBlock][kMaxSteps + 1];
  __shared__ double s_lds[kBlock];
  __shared__ double wsum[4][kMaxSteps];
  __shared__ double rmin[kBlock / kMaxSteps][kMaxSteps];
  const int kc = blockIdx.x, gcb = blockIdx.y;
  const int TM = a.T * a.m;
  const int chunk = a.upd_chunk, ppt = chunk / kUpdStrips;
  const uint64_t it = *a.iter;
  const int f_lo = gcb * kUpdGroups * 4, f_hi = min(f_lo + kUpdGroups * 4, TM);
  const int i_lo = (f_lo + a.m - 1) / a.m, n_i = (f_hi + a.m - 1) / a.m - i_lo;
  // weights and normalisers of those steps (prefix costs and minima loaded up front)
  {
    const int k = kc * chunk + threadIdx.x;
    const bool in = (int)threadIdx.x < chunk && k < a.K;
    const double s = in ? a.S[k] : __builtin_inf();
    double tail[kMaxSteps], rho_i[kMaxSteps];
#pragma unroll
    for (int j = 0; j < kMaxSteps; ++j) tail[j] = in && j < n_i ? a.pre[(size_t)(i_lo + j) * a.K + k] : 0.0;
    if (a.blk_tail) {
      // the per-step minima from the rollout blocks' own: thread (q, j) reduces blocks
      // q, q + 16, ... of step i_lo + j, then the sixteen partial minima (min is exact, so the
      // order does not matter); kc = 0 stores them for the finalize
      constexpr int NQ = kBlock / kMaxSteps;
      const int q = threadIdx.x % NQ, j = threadIdx.x / NQ;      // sixteen threads per step: coalesced
      static_assert(kBlock / NQ == kMaxSteps, "one thread row per step");
      double m = __builtin_inf();
      if (j < n_i) {
        const double *row = a.blk_tail + (size_t)(i_lo + j) * a.n_roll_blocks;
        constexpr int kB = 16;                      // loads in flight per round
        for (int b0 = q; b0 < a.n_roll_blocks; b0 += NQ * kB) {
          double v[kB];
#pragma unroll
          for (int u = 0; u < kB; ++u) {
            const int b = b0 + NQ * u;
            v[u] = b < a.n_roll_blocks ? row[b] : __builtin_inf();
          }
#pragma unroll
          for (int u = 0; u < kB; ++u) m = fmin(m, v[u]);
        }
      }
      rmin[q][j] = m;
      __syncthreads();
      if ((int)threadIdx.x < n_i) {
        double r = rmin[0][threadIdx.x];
        for (int qq = 1; qq < NQ; ++qq) r = fmin(r, rmin[qq][threadIdx.x]);
        rmin[0][threadIdx.x] = r;
        if (kc == 0) a.rho_step[i_lo + threadIdx.x] = r;
      }
      __syncthreads();
#pragma unroll
      for (int jj = 0; jj < kMaxSteps; ++jj) rho_i[jj] = jj < n_i ? rmin[0][jj] : 0.0;
    } else {
#pragma unroll
      for (int jj = 0; jj < kMaxSteps; ++jj) rho_i[jj] = jj < n_i ? a.rho_step[i_lo + jj] : 0.0;
    }
    s_lds[threadIdx.x] = s;
    // the steps' block sums (each in block_sum's order) share one barrier; thread j
    // writes step i_lo + j
    const int wv = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < kMaxSteps; ++j) {
      if (j < n_i) {
        const double w = s < __builtin_inf() ? exp(-((s - tail[j]) - rho_i[j]) * a.inv_lambda) : 0.0;
        w_lds[threadIdx.x][j] = w;
        const double ws = wave_sum(w);
        if ((threadIdx.x & (kWave - 1)) == 0) wsum[wv][j] = ws;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < n_i) {
      const int j = threadIdx.x;
      a.eta_part[(size_t)kc * a.T + i_lo + j] = (wsum[0][j] + wsum[1][j]) + (wsum[2][j] + wsum[3][j]);
    }
  }
  const int gl = threadIdx.x % kUpdGroups, strip = threadIdx.x / kUpdGroups;
  const int g = gcb * kUpdGroups + gl;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (g < a.G) {
    for (int r = 0; r < ppt; ++r) {
      const int kl = strip * ppt + r;
      if (s_lds[kl] < __builtin_inf()) {
        float e[4];
        normals4((uint32_t)g, (uint32_t)(kc * chunk + kl), it, a.key0, a.key1, e);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int f = 4 * g + c;
          if (f < TM) acc[c] = fma(w_lds[kl][f / a.m - i_lo], (double)e[c], acc[c]);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) acc_lds[strip][gl][c] = acc[c];
  __syncthreads();
  {
    const int slot = threadIdx.x % (kUpdGroups * 4), run = threadIdx.x / (kUpdGroups * 4);
    if (run < 16) {
      const int gg = slot / 4, c = slot % 4;
      double s = 0.0;
      for (int st = run * (kUpdStrips / 16); st < (run + 1) * (kUpdStrips / 16); ++st) s += acc_lds[st][gg][c];
      runs[run][slot] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < kUpdGroups * 4) {
    const int gg = threadIdx.x / 4, c = threadIdx.x % 4;
    const int gabs = gcb * kUpdGroups + gg;
    double s = 0.0;
    for (int r = 0; r < 16; ++r) s += runs[r][threadIdx.x];
    if (gabs < a.G) a.part[(size_t)kc * (a.G * 4) + gabs * 4 + c] = s;
  }
}

// ----------------------------------------------------------------------- finalize
// One block of 1024 threads; T*m <= 4096 handled in a strided loop.  Sums over the
// chunk partials run in a fixed order (c = 0, 1, ...) with their loads issued 32 at
// a time, so the result is independent of timing and of the batch it runs in.
constexpr int kFinBlock = 1024;
constexpr int kMaxTM = 4096;

__device__ __forceinline__ double ordered_sum(const double *p, size_t stride, int n) {
  constexpr int kBatch = 32;                       // loads in flight per round
  double s = 0.0;
  int c = 0;
  for (; c + kBatch <= n; c += kBatch) {
    double v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) v[j] = p[(size_t)(c + j) * stride];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) s += v[j];
  }
  if (c < n) {
    double v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) v[j] = c + j < n ? p[(size_t)(c + j) * stride] : 0.0;
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (c + j < n) s += v[j];
  }
  return s;
}

// status_out (nullable): 0 when the iteration had a finite cost, -5 otherwise.  The
// minimum comes from the update (every update block reduces the block minima anyway); all
// global loads (chunk partials, the previous sequence) are issued before the first
// barrier; the updated sequence then lives in LDS until the (shifted) write-back.
// Returns with u0 (the emitted control, when a.emit) in u0_s.
__device__ __forceinline__ void finalize_body(const FinalizeArgs &a, double *u0_out, double *status_out,
                                              double *u0_s) {
  constexpr int NT = kFinBlock;
  __shared__ double N_lds[kMaxTM];
  __shared__ double eta_step[1024];                // per-step normalisers (cost-to-go weights)
  __shared__ double eta_s;
  constexpr int kPer = kMaxTM / NT;
  const int TM = a.T * a.m;
  const double rho = *a.rho;
  const uint64_t it0 = threadIdx.x == 0 ? a.iter[0] : 0;   // loaded with the rest, not after
  double Uold[kPer];
#pragma unroll
  for (int n = 0; n < kPer; ++n) {
    const int f = threadIdx.x + n * NT;
    Uold[n] = f < TM ? a.U64[f] : 0.0;
  }
  if (a.ctg) {
    for (int i = threadIdx.x; i < a.T; i += NT) eta_step[i] = ordered_sum(a.eta_part + i, (size_t)a.T, a.n_kc);
  } else if (threadIdx.x == 0) {
    eta_s = ordered_sum(a.eta_part, 1, a.n_kc);
  }
  for (int f = threadIdx.x; f < TM; f += NT) N_lds[f] = ordered_sum(a.part + f, (size_t)a.G * 4, a.n_kc);
  __syncthreads();
  const bool ok = rho < __builtin_inf();
  const double eta = a.ctg ? eta_step[0] : eta_s;
  const double inv_eta = ok ? 1.0 / eta : 0.0;
  double Unew[kPer];
#pragma unroll
  for (int n = 0; n < kPer; ++n) {
    const int f = threadIdx.x + n * NT;
    Unew[n] = Uold[n];
    if (f < TM) {
      const int i = f / a.m, j = f - i * a.m;
      double d = 0.0;
      for (int l = 0; l <= j; ++l) d = fma(a.Ls[j * a.m + l], N_lds[i * a.m + l], d);
      d = ok ? d * (a.ctg ? 1.0 / eta_step[i] : inv_eta) : 0.0;
      a.dbg[2 + f] = d;
      Unew[n] = Uold[n] + d;
    }
  }
  if (threadIdx.x == 0) {
    a.dbg[0] = rho;
    a.dbg[1] = ok ? eta : 0.0;
    if (!ok) a.flags[0] += 1;
    if (status_out) *status_out = ok ? 0.0 : -5.0;
    a.iter[0] = it0 + 1;
  }
  if (a.emit) {
    __syncthreads();                                   // everyone has read N_lds
#pragma unroll
    for (int n = 0; n < kPer; ++n) {
      const int f = threadIdx.x + n * NT;
      if (f < TM) N_lds[f] = Unew[n];
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < kPer; ++n) {
      const int f = threadIdx.x + n * NT;
      if (f < a.m) {
        u0_out[f] = N_lds[f];
        u0_s[f] = N_lds[f];
      }
      if (f < TM) Unew[n] = (f + a.m < TM) ? N_lds[f + a.m] : a.u_init[f - (TM - a.m)];
    }
    __syncthreads();
  }
#pragma unroll
  for (int n = 0; n < kPer; ++n) {
    const int f = threadIdx.x + n * NT;
    if (f < TM) {
      a.U64[f] = Unew[n];
      a.U32[f] = (float)Unew[n];
    }
  }
}

static __global__ __launch_bounds__(kFinBlock) void finalize_kernel(const FinalizeArgs a) {
  __shared__ double u0_s[4];
  finalize_body(a, a.u0_out, nullptr, u0_s);
}

// Multi-block finalize, block fb of ceil(T*m / kFinOut): components [4 fb, 4 fb + 4), whole
// time steps since m divides 4.  Every block forms rho = min_b rho_b, the factors
// alpha_b = exp(-(rho_b - rho)/lambda) and eta = sum_b alpha_b eta_b from the same loads in
// the same order, so all agree bit for bit.  Under cost-to-go weighting each of the block's
// steps i has its own: rho_i = min_b rho_b,i (the rollout blocks' per-step minima), alpha_b,i
// and eta_i = sum_b alpha_b,i eta_b,i, and a component is rescaled and normalised by those
// of its step (the block's first step's minimum is finite exactly when some path cost is).  Thread (r, c) = (t / 4, t % 4) sums
// alpha_b N_b,c over the rollout blocks b = r + 256 j in order of j; the sixteen runs of a
// wave that share c are added by a butterfly, then the sixteen waves' sums in order.  The old
// sequence comes from the shadow the rollout wrote, so the shifted write-back into U64 cannot
// race with another block's read.  Block 0 emits u0, counts the iteration and writes the
// diagnostics.  `after_loads` runs once the loads are issued, before the first barrier.
// Returns with u0 in u0_s (block 0, when a.emit).
// kSteps: 1 under path weighting, kFinOut (the most steps a block holds, m = 1) under
// cost-to-go weighting; the kernels pick the instance from a.ctg.  A finalize block is
// kFinMultiBlock threads; kSub of them share a workgroup (the batched server's 1024-thread
// blocks hold four: each runs the same code on its own LDS, and every barrier is taken by all
// four together), so a controller's results do not depend on how its blocks are packed.
// Thread t of a block loads the minima and normalisers of rollout blocks t, t + 256, ...
// and sums its share of the weighted normalisers in that order before the wave sums.
template <int kSteps, int kSub, class Hook>
__device__ __forceinline__ void finalize_multi_body(const FinalizeArgs &a, int fb, double *u0_out,
                                                    double *status_out, double *u0_s, Hook after_loads) {
  constexpr int NT = kFinMultiBlock, NR = NT / kFinOut, NW = NT / kWave, kPerRun = kMaxMergedParts / NR;
  constexpr int U = kMaxMergedParts / NT;             // rollout blocks per thread for the minima
  static_assert(kFinOut % 4 == 0 && kWave % kFinOut == 0 && kPerRun >= 1 && U >= 1, "multi-block finalize layout");
  static_assert(kSteps == 1 || kSteps == kFinOut, "one step or a block's worth");
  __shared__ double alpha_all[kSub][kSteps][kMaxMergedParts];   // per step
  __shared__ double wsum_all[kSub][NW][kFinOut];
  __shared__ double N_all[kSub][kFinOut];
  __shared__ double red_all[kSub][NW];
  const int sub = kSub > 1 ? (int)threadIdx.x / NT : 0;
  const int lt = kSub > 1 ? (int)threadIdx.x % NT : (int)threadIdx.x;
  double (*alpha)[kMaxMergedParts] = alpha_all[sub];
  double (*wsum)[kFinOut] = wsum_all[sub];
  double *N_s = N_all[sub], *red = red_all[sub];
  const int TM = a.T * a.m, P = a.n_parts, F = a.G * 4;
  const int c = lt % kFinOut, r = lt / kFinOut;
  const int f = fb * kFinOut + c;
  const int i0 = fb * kFinOut / a.m;                  // the block's first step
  const int ns = kSteps > 1 ? min(kFinOut / a.m, a.T - i0) : 1;
  // every load up front: block minima and normalisers (U each per thread and step), this
  // thread's partials, the old sequence and its row of A chol(Sigma), the counter
  double mb[kSteps][U], eb[kSteps][U];
#pragma unroll
  for (int st = 0; st < kSteps; ++st)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = lt + NT * u;
      const bool in = st < ns && b < P;
      if constexpr (kSteps > 1) {
        mb[st][u] = in ? a.blk_tail[(size_t)(i0 + st) * P + b] : __builtin_inf();
        eb[st][u] = in ? a.eta_part[(size_t)b * a.T + i0 + st] : 0.0;
      } else {
        mb[st][u] = in ? a.blk_min[b] : __builtin_inf();
        eb[st][u] = in ? a.eta_part[b] : 0.0;
      }
    }
  double pv[kPerRun];
#pragma unroll
  for (int j = 0; j < kPerRun; ++j) {
    const int b = r + NR * j;
    pv[j] = b < P && f < TM ? a.part[(size_t)b * F + f] : 0.0;
  }
  const bool owner = r == 0 && f < TM;
  const int i = f / a.m, jc = f - i * a.m;
  const double Uold = owner ? a.Ushadow[f] : 0.0;
  double Lrow[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) Lrow[l] = owner && l <= jc ? a.Ls[jc * a.m + l] : 0.0;
  const uint64_t it0 = fb == 0 && lt == 0 ? a.iter[0] : 0;
  after_loads();
  // each step's minimum, factors and normaliser (a reduction pair per step)
  double rho[kSteps], eta[kSteps];
#pragma unroll
  for (int st = 0; st < kSteps; ++st) {
    rho[st] = __builtin_inf();
    eta[st] = 0.0;
    if (st < ns) {                                    // uniform over the workgroup
      double m = mb[st][0];
#pragma unroll
      for (int u = 1; u < U; ++u) m = fmin(m, mb[st][u]);
      m = wave_min(m);
      __syncthreads();
      if ((lt & (kWave - 1)) == 0) red[lt / kWave] = m;
      __syncthreads();
      double rr = red[0];
#pragma unroll
      for (int w = 1; w < NW; ++w) rr = fmin(rr, red[w]);
      rho[st] = rr;
      double e = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double al = rr < __builtin_inf() && mb[st][u] < __builtin_inf()
                              ? exp(-(mb[st][u] - rr) * a.inv_lambda) : 0.0;
        alpha[st][lt + NT * u] = al;                  // 0 past the last block
        e = fma(al, eb[st][u], e);
      }
      e = wave_sum(e);
      __syncthreads();                                // also publishes alpha
      if ((lt & (kWave - 1)) == 0) red[lt / kWave] = e;
      __syncthreads();
      double es = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) es += red[w];
      eta[st] = es;
    }
  }
  const int sc = kSteps > 1 && f < TM ? f / a.m - i0 : 0;   // this component's step in the block
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < kPerRun; ++j) acc = fma(alpha[sc][r + NR * j], pv[j], acc);
  // the wave's runs of component c (lanes c + kFinOut q) by an xor butterfly: partners
  // add the same two values, so every lane ends with the same bits
#pragma unroll
  for (int st = kFinOut; st < kWave; st *= 2) acc += __shfl_xor(acc, st);
  if ((lt & (kWave - 1)) < kFinOut) wsum[lt / kWave][c] = acc;
  __syncthreads();
  if (lt < kFinOut) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += wsum[w][lt];
    N_s[lt] = sum;
  }
  __syncthreads();
  const bool ok = rho[0] < __builtin_inf();
  if (owner) {
    const int base = i * a.m - fb * kFinOut;
    double eta_c = eta[0];                            // this component's step's normaliser
#pragma unroll
    for (int st = 1; st < kSteps; ++st)
      if (st == sc) eta_c = eta[st];
    const double inv_eta = ok ? 1.0 / eta_c : 0.0;
    double d = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
      if (l <= jc) d = fma(Lrow[l], N_s[base + l], d);
    d = ok ? d * inv_eta : 0.0;
    a.dbg[2 + f] = d;
    const double Unew = Uold + d;
    if (!a.emit) {
      a.U64[f] = Unew;
      a.U32[f] = (float)Unew;
    } else {
      if (f < a.m) {
        u0_out[f] = Unew;
        u0_s[f] = Unew;
      } else {
        a.U64[f - a.m] = Unew;
        a.U32[f - a.m] = (float)Unew;
      }
      if (f >= TM - a.m) {
        a.U64[f] = a.u_init[f - (TM - a.m)];
        a.U32[f] = (float)a.u_init[f - (TM - a.m)];
      }
    }
  }
  if (kSteps > 1 && lt == 0) {
#pragma unroll
    for (int st = 0; st < kSteps; ++st)
      if (st < ns) a.rho_step[i0 + st] = rho[st];
  }
  if (fb == 0 && lt == 0) {
    a.dbg[0] = rho[0];
    a.dbg[1] = ok ? eta[0] : 0.0;
    if (!ok) a.flags[0] += 1;
    if (status_out) *status_out = ok ? 0.0 : -5.0;
    a.iter[0] = it0 + 1;
  }
  if (a.emit) __syncthreads();                        // u0_s for the plant step
}

static __global__ __launch_bounds__(kFinMultiBlock) void finalize_multi_kernel(const FinalizeArgs a) {
  __shared__ double u0_s[4];
  if (a.ctg) finalize_multi_body<kFinOut, 1>(a, blockIdx.x, a.u0_out, nullptr, u0_s, [] {});
  else finalize_multi_body<1, 1>(a, blockIdx.x, a.u0_out, nullptr, u0_s, [] {});
}

// finalize + the plant step on the emitted control.  The last wave evaluates the plant
// basis: it owns no sequence component while T*m <= kFinBlock - 64, so the basis overlaps
// the other waves' loads instead of delaying them.
template <class Sys>
__global__ __launch_bounds__(kFinBlock) void finalize_plant_kernel(const FinalizeArgs a, double *x, double dt, int n,
                                                                   const typename Sys::Params p) {
  __shared__ double u0_s[4];
  __shared__ double basis[Sys::M + 1][Sys::N];
  const int j = (int)threadIdx.x - (kFinBlock - kWave);
  if (j >= 0 && j <= Sys::M) plant_basis<Sys>(p, x, n, j, basis[j]);
  finalize_body(a, a.u0_out, nullptr, u0_s);          // its barriers publish the basis
  if (threadIdx.x == 0) plant_combine<Sys>(x, n, dt, basis, u0_s);
}

// The multi-block finalize + the plant step: block 0, which emits u0, combines it with the
// plant basis the rollout's extra block wrote; no other block touches x.
template <class Sys>
__global__ __launch_bounds__(kFinMultiBlock) void finalize_multi_plant_kernel(const FinalizeArgs a, double *x,
                                                                              double dt, int n, const double *basis) {
  __shared__ double u0_s[4];
  if (a.ctg) finalize_multi_body<kFinOut, 1>(a, blockIdx.x, a.u0_out, nullptr, u0_s, [] {});
  else finalize_multi_body<1, 1>(a, blockIdx.x, a.u0_out, nullptr, u0_s, [] {});
  if (blockIdx.x == 0 && threadIdx.x == 0)
    plant_combine<Sys>(x, n, dt, reinterpret_cast<const double (*)[Sys::N]>(basis), u0_s);
}

// The plant step alone (block of one wave).
template <class Sys>
__global__ void plant_kernel(double *x, const double *u, double dt, int n, const typename Sys::Params p) {
  __shared__ double basis[Sys::M + 1][Sys::N];
  if (threadIdx.x <= Sys::M) plant_basis<Sys>(p, x, n, threadIdx.x, basis[threadIdx.x]);
  __syncthreads();
  if (threadIdx.x == 0) plant_combine<Sys>(x, n, dt, basis, u);
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

// The lane-group helpers of the rollouts on one full wave per block (every lane active,
// as in the rollouts): per lane, the inclusive and exclusive scans of a, the broadcast
// of the group's last lane, the FP64 group sum (meaningful in the group's first lane)
// and, for G <= 16, the inclusive scan of the affine maps x -> a x + b.
template <int G>
static __global__ __launch_bounds__(kWave) void lane_groups_kernel(const float *a_in, const float *b_in, float *out) {
  const int t = blockIdx.x * kWave + threadIdx.x;
  const int lj = threadIdx.x % G;
  const float a = a_in[t], b = b_in[t];
  const float incl = group_scan_incl<G>(a, lj);
  out[6 * t + 0] = incl;
  out[6 * t + 1] = group_excl_of_incl<G>(incl, lj);
  out[6 * t + 2] = group_bcast<G, G - 1>(a);
  out[6 * t + 3] = (float)group_sum<G>((double)a);
  float A = a, B = b;
  if constexpr (G <= 16) {
    group_affine_scan_incl<G>(A, B, lj);
  } else {
    A = B = __builtin_nanf("");
  }
  out[6 * t + 4] = A;
  out[6 * t + 5] = B;
}

}  // namespace mppi
