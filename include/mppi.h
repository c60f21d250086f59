/*
 * mppi.h -- C ABI of libmppi: Model Predictive Path Integral control with
 * covariance-variable importance sampling on AMD Instinct MI355X (gfx950).
 *
 * Method: Williams, Aldrich & Theodorou, "Model Predictive Path Integral Control
 * using Covariance Variable Importance Sampling" (arXiv 1509.01149).
 *   - problem statement (control-affine dynamics, state cost q, terminal cost phi,
 *     control cost R): Section II;
 *   - likelihood-ratio running cost for the special case A = sqrt(nu) I and the
 *     Monte-Carlo update law: Section III-C; a diagonal covariance change
 *     A = diag(sqrt(nu_j)) from the theorem of Section III-A (mppi_config.nu_diag);
 *   - the control loop (sample, roll out, weight, update, send u0, shift, u_init):
 *     Algorithm 1, Section IV;
 *   - the experiments' swing-up cart-pole and the quadrotor's crash indicator:
 *     Section V.
 *
 * Conventions for every function below:
 *   - Every call returns an mppi_status; nothing throws across the ABI.  On failure
 *     mppi_last_error() returns a thread-local message describing the first error.
 *   - Host arrays passed in are owned by the caller and copied before the call
 *     returns; the library never keeps or frees a caller pointer, except a lent
 *     workspace (mppi_config.workspace), which must outlive the context.
 *   - Matrices are row-major, FP64 on the host.  The library rounds to FP32 where the
 *     rollouts need it and keeps the nominal control sequence, the weights'
 *     normaliser and the weighted update in FP64 on the device.
 *   - A context is used by one host thread at a time and runs its work in order on
 *     its stream.  A server (mppi_server_*) is internally synchronised.
 *   - "Device pointer" means memory on the context's device (hipMalloc or a torch
 *     CUDA tensor); "host pointer" means ordinary or pinned host memory.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_ABI_VERSION 1

typedef enum {
  MPPI_OK = 0,
  MPPI_EINVAL = -1,    /* invalid argument or configuration; nothing was changed      */
  MPPI_ENOMEM = -2,    /* device or host allocation failed, or workspace too small    */
  MPPI_EDEVICE = -3,   /* a HIP call failed or no usable GPU is present               */
  MPPI_EBUSY = -4,     /* server: no slot or HBM budget free right now; retry later   */
  MPPI_ENUMERIC = -5,  /* every sample of some iteration had a non-finite path cost:  */
                       /* that iteration left the control sequence unchanged          */
  MPPI_ENOTFOUND = -6  /* server: unknown slot or request                             */
} mppi_status;

/* Compiled-in systems.  The dynamics f, G and the costs q, phi of Section II cannot be
 * host callbacks on a GPU, so they are chosen from this registry and parameterised by
 * the matching mppi_*_params block passed in mppi_config.params. */
typedef enum {
  MPPI_SYS_LINEAR = 0,        /* x' = A x + B u,  q = x'Qx, phi = x'Qf x         */
  MPPI_SYS_CARTPOLE = 1,      /* cart with uniform pole, force input             */
  MPPI_SYS_BICYCLE = 2,       /* kinematic bicycle on a bilinear cost map        */
  MPPI_SYS_QUADROTOR = 3,     /* 12-state rigid-body quadrotor, spherical obstacles */
  MPPI_SYS_QUADROTOR_MLP = 4, /* quadrotor cost, dynamics by a learned MLP (mppi_mlp) */
  MPPI_SYS_CARTPOLE_SWINGUP = 5 /* velocity-command cart-pole of the swing-up task    */
} mppi_system;

/* MPPI_SYS_LINEAR: n_state <= 4, n_ctrl in {1, 2, 4}.  A (n x n), B (n x m), Q (n x n),
 * Qf (n x n), all row-major FP64, copied at create. */
typedef struct {
  const double *A, *B, *Q, *Qf;
} mppi_linear_params;

/* MPPI_SYS_CARTPOLE: state (x, xdot, theta, thetadot), theta = 0 upright, n = 4, m = 1.
 *   h = (F + mp l thetadot^2 sin theta) / (mc + mp)
 *   thetaddot = (g sin theta - cos theta h) / (l (4/3 - mp cos^2 theta / (mc + mp)))
 *   xddot = h - mp l thetaddot cos theta / (mc + mp)
 * q(x) = sum_i q_diag[i] x_i^2, phi(x) = sum_i qf_diag[i] x_i^2. */
typedef struct {
  double mass_cart, mass_pole, half_length, gravity;
  double q_diag[4];
  double qf_diag[4];
} mppi_cartpole_params;

/* MPPI_SYS_CARTPOLE_SWINGUP (Section V-A): state (p, pdot, theta, thetadot), theta = 0
 * hanging down, theta = pi upright, n = 4, m = 1; the control is a desired cart velocity.
 * pddot = gain (u - pdot); thetaddot = -(3 / (4 l)) (g sin theta + pddot cos theta)
 * (uniform pole of half-length l on the accelerated pivot).
 * q = w_pos p^2 + w_angle (1 + cos theta)^2 + w_rate thetadot^2 + w_vel pdot^2, phi = 0. */
typedef struct {
  double gain, half_length, gravity;
  double w_pos, w_angle, w_vel, w_rate;
} mppi_swingup_params;

/* MPPI_SYS_BICYCLE: state (x, y, yaw, v, delta), controls (accel, steer rate), n = 5, m = 2.
 *   x' = v cos yaw, y' = v sin yaw, yaw' = v tan(clamp(delta, +-steer_limit)) / wheelbase,
 *   v' = a, delta' = omega   (steer_limit <= 0: no clamp)
 * q = bilinear(map, x / cell_size, y / cell_size) + w_speed (v - v_target)^2, phi = 0.
 * The map is map_h x map_w FP32, row-major [y][x], cell (0,0) centred at the origin,
 * coordinates clamped to the grid; copied at create.  map_w, map_h >= 2. */
typedef struct {
  double wheelbase, v_target, w_speed, cell_size, steer_limit;
  int32_t map_w, map_h;
  const float *map;
} mppi_bicycle_params;

/* MPPI_SYS_QUADROTOR: state (p[3], v[3], roll, pitch, yaw, body rates w[3]), n = 12,
 * controls = rotor thrusts (f1 on +x, f2 on +y, f3 on -x, f4 on -y), m = 4.
 *   p' = v,  v' = (sum f / mass) R_zyx(roll, pitch, yaw) e3 - gravity e3,
 *   euler' = W(euler)^-1 w,  w' = J^-1 (tau - w x J w),
 *   tau = (arm (f2 - f4), arm (f3 - f1), yaw_coef (f1 - f2 + f3 - f4)),  J = diag(inertia)
 * q = w_goal |p - goal|^2 + w_obs sum_j max(0, (r_j + obs_margin)^2 - |p - c_j|^2)^2,
 * phi = 0.  obstacles: n_obstacles x 4 (cx, cy, cz, r) FP64, copied; n_obstacles <= 256;
 * finite centres, r >= 0 and r + obs_margin <= 1e6, obs_margin >= 0, w_obs in [0, 1e12]
 * (else MPPI_EINVAL).
 * crash_cost > 0 adds the crash indicator C (Section V-C): C = 1 once p_z < ground_z or
 * |p - c_j| < r_j; from then on the rollout stops simulating, the vehicle stays where it
 * is and every remaining step adds crash_cost (not with MPPI_SYS_QUADROTOR_MLP). */
typedef struct {
  double mass, gravity, arm, yaw_coef;
  double inertia[3];
  double goal[3];
  double w_goal, w_obs, obs_margin;
  int32_t n_obstacles;
  const double *obstacles;
  double crash_cost;          /* crash indicator C (Section V-C); 0 disables it          */
  double ground_z;            /* ground plane height for C                               */
} mppi_quadrotor_params;

/* MPPI_SYS_QUADROTOR_MLP: the quadrotor's cost with dynamics x <- x + MLP(x, u)
 * (an mppi_mlp, see "Learned dynamics" below).  Its current parameters and statistics
 * are copied at create; the harness plant (mppi_plant_step_async) stays analytic. */
typedef struct mppi_mlp mppi_mlp;
typedef struct {
  mppi_quadrotor_params quad;
  const mppi_mlp *mlp;
} mppi_quadrotor_mlp_params;

/* Everything Algorithm 1 is "given" (Section IV), plus device placement. */
typedef struct {
  int32_t abi_version;        /* must be MPPI_ABI_VERSION                                  */
  int32_t system;             /* mppi_system                                               */
  int32_t n_state, n_ctrl;    /* n, m; must match the system                               */
  int32_t K;                  /* samples (rollouts) per iteration, 1 <= K <= 4194304        */
  int32_t T;                  /* horizon steps N of Algorithm 1, 1 <= T <= 1024            */
  double dt;                  /* time step of the Euler discretisation (Section II-A)      */
  double lambda;              /* temperature, > 0                                          */
  double nu;                  /* exploration factor: perturbations ~ N(0, nu Sigma), > 0;  */
                              /* the paper's experiments use nu >= 1                      */
  const double *sigma;        /* m x m natural per-step covariance of the perturbation     */
  const double *R;            /* m x m control-cost matrix; NULL => lambda * inv(sigma)    */
  const double *u_init;       /* m: value of the control appended by the warm shift        */
  const double *u_nominal0;   /* T x m initial nominal sequence; NULL => u_init repeated   */
  const void *params;         /* the system's mppi_*_params block                          */
  uint64_t params_bytes;      /* sizeof that block                                         */
  uint64_t seed;              /* Philox4x32-10 key of the rollout noise                    */
  int32_t device;             /* HIP device ordinal                                        */
  int32_t use_graph;          /* nonzero: replay each step as a captured hipGraph, one per */
                              /* (n_iters, device pointers) combination, at most 16 kept  */
  void *stream;               /* hipStream_t to run on; NULL => the library makes its own  */
  void *workspace;            /* optional caller-owned device memory for all device state  */
  uint64_t workspace_bytes;   /* its size; must be >= mppi_workspace_bytes()               */
  const double *nu_diag;      /* m per-dimension exploration factors (a diagonal covariance */
                              /* change A = diag(sqrt(nu_j)), Section III-A); NULL => nu.   */
                              /* The quadratic likelihood-ratio term becomes               */
                              /* du'(R - A^-1 R A^-1) du / 2; copied                       */
  int32_t weighting;          /* MPPI_WEIGHT_PATH or MPPI_WEIGHT_COST_TO_GO                */
  int32_t kernels;            /* MPPI_KERNELS_AUTO (0), _FUSED or _THREE                   */
} mppi_config;

/* Kernels per iteration.  THREE: rollout, update (regenerates the noise to form the weighted
 * sums), finalize.  FUSED: the rollout keeps its block's normals in LDS and also forms the
 * weighted sums of its samples, and the finalize merges them (MPPI_ROLLOUT_FUSED; with at
 * most 1024 rollout blocks and a block's normals within its LDS: 32 KiB on the step-split
 * systems, which under cost-to-go weighting also keep their samples' running costs, at most
 * 32 KiB; on the quadrotor, under path weighting only, the rest of a 160 KiB CU, 64 samples
 * x T*4 floats, so T <= 153 with 32 obstacles; else MPPI_EINVAL).  AUTO takes FUSED wherever it is
 * available, on the quadrotor only while its rollout blocks (64 samples each) number at
 * most 256, one per CU of an MI355X (K <= 16384).  Both compute the update law of
 * Section III-C; their results differ by FP64 summation order only. */
enum { MPPI_KERNELS_AUTO = 0, MPPI_KERNELS_FUSED = 2, MPPI_KERNELS_THREE = 3 };

/* Weights of the update law (Section III-C).  PATH: one total path cost per sample weights
 * every time step (Algorithm 1's forward-accumulated cost).  COST_TO_GO: time step i is
 * weighted by each sample's cost from step i onward, as the update law's S(tau_{i,k}) reads,
 * with a per-step minimum and normaliser; it adds T x K FP64 of workspace and is not
 * available with MPPI_SYS_QUADROTOR_MLP or through the server (MPPI_EINVAL). */
enum { MPPI_WEIGHT_PATH = 0, MPPI_WEIGHT_COST_TO_GO = 1 };

typedef struct mppi_ctx mppi_ctx;

/* Bytes of device memory a context for cfg needs (to size a lent workspace). */
int mppi_workspace_bytes(const mppi_config *cfg, uint64_t *bytes);

/* Validate cfg, copy its arrays, allocate (or carve the lent workspace into) device
 * buffers and upload the nominal sequence.  The iteration counter starts at 0. */
int mppi_create(const mppi_config *cfg, mppi_ctx **out);

/* Wait for the context's work and free everything it owns.  NULL is accepted. */
int mppi_destroy(mppi_ctx *ctx);

/* One control step of Algorithm 1 from state x0 (host, n): n_iters >= 1 iterations of
 * {sample, roll out, weight, update}, then write u0 = u_0 (host, m) and shift the
 * sequence (u_i <- u_{i+1}, u_{T-1} <- u_init).  Blocks until done.
 * Returns MPPI_ENUMERIC if some iteration had no finite path cost (u0 and the shift are
 * still produced). */
int mppi_step(mppi_ctx *ctx, const double *x0, int32_t n_iters, double *u0);

/* As mppi_step with device pointers x0_dev (n FP64) and u0_dev (m FP64), enqueued on
 * the context's stream; returns without waiting.  The numeric status is collected by
 * mppi_sync. */
int mppi_step_async(mppi_ctx *ctx, const double *x0_dev, int32_t n_iters, double *u0_dev);

/* Closed-loop form of mppi_step_async for simulation on the device: x_dev (n FP64) is the
 * start state of the step and, once u0 is emitted into u0_dev (m FP64), is advanced by the
 * harness plant step (as mppi_plant_step_async) inside the same launch sequence. */
int mppi_step_plant_async(mppi_ctx *ctx, double *x_dev, int32_t n_iters, double *u0_dev);

/* n_steps consecutive closed-loop steps on the device in one launch sequence (one
 * captured graph when use_graph is set): exactly n_steps calls of mppi_step_plant_async
 * with u0_dev = u_log_dev + j m for step j (the same results bit for bit), without the
 * per-launch gap between steps.  u_log_dev holds n_steps x m FP64 (device).
 * 1 <= n_steps, n_iters and n_steps * n_iters <= 1000; status collected by mppi_sync. */
int mppi_run_closed_loop_async(mppi_ctx *ctx, double *x_dev, int32_t n_steps, int32_t n_iters, double *u_log_dev);

/* Wait for the context's stream.  Returns MPPI_ENUMERIC if any iteration since the
 * previous mppi_sync / mppi_step had no finite path cost, and clears that flag. */
int mppi_sync(mppi_ctx *ctx);

/* Harness plant (Algorithm 1: "update the current state after receiving feedback"):
 * x_dev <- x_dev + dt (f(x) + G(x) u_dev) in FP64 with the context's model, no noise.
 * Device pointers, enqueued on the context's stream. */
int mppi_plant_step_async(mppi_ctx *ctx, double *x_dev, const double *u_dev);

/* Allocation-free control step, for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc).  It computes exactly
 * what mppi_create(cfg) with u_nominal0 = U and the iteration counter at *iteration, followed
 * by mppi_step(ctx, x0, n_iters, u0) and mppi_get_controls, would: the same kernels on the same
 * inputs, so the results are bit for bit those of that sequence.  The caller holds the
 * controller state between calls:
 *   x0         host, n       start state
 *   U          host, T x m   in: nominal sequence; out: the sequence after the update and the
 *                            warm shift (u_i <- u_{i+1}, u_{T-1} <- u_init)
 *   iteration  host, 1       in: noise counter; out: advanced by n_iters
 *   u0         host, m       out: the control sent to the actuators
 * Every device buffer of the step (path costs, partial sums, the FP32 sequence, the cost map
 * or obstacles) lives in one static device array of MPPI_STATIC_SCRATCH_BYTES per GPU, which
 * the library keeps until the process ends; the call makes no device or pinned allocation.
 * It runs on cfg->stream (NULL: the null stream) and blocks until done; cfg->workspace and
 * cfg->use_graph are ignored.  All calls on one GPU share that array: calls that overlap on
 * one GPU (from several threads) race and must be serialised by the caller.
 * Errors: MPPI_EINVAL for an invalid cfg or argument, for MPPI_SYS_QUADROTOR_MLP, and when the
 * step needs more than MPPI_STATIC_SCRATCH_BYTES (the same bytes mppi_workspace_bytes reports);
 * MPPI_ENUMERIC as for mppi_step (u0 and the shift are still produced); MPPI_EDEVICE. */
#define MPPI_STATIC_SCRATCH_BYTES (8ull << 20)
int mppi_step_static(const mppi_config *cfg, const double *x0, double *U, uint64_t *iteration, int32_t n_iters,
                     double *u0);

/* Copy the current (post-shift) nominal sequence, T x m FP64, to / from the host. */
int mppi_get_controls(mppi_ctx *ctx, double *u, uint64_t len);
int mppi_set_controls(mppi_ctx *ctx, const double *u, uint64_t len);

/* Snapshot / restore of the controller state: the FP64 nominal sequence and the
 * iteration counter that keys the noise.  buf is host memory of *needed bytes
 * (query with buf = NULL). */
int mppi_get_state(mppi_ctx *ctx, void *buf, uint64_t len, uint64_t *needed);
int mppi_set_state(mppi_ctx *ctx, const void *buf, uint64_t len);
int mppi_get_iteration(mppi_ctx *ctx, uint64_t *iteration);

/* Diagnostics of the last iteration (host outputs; any pointer may be NULL):
 * path costs S-tilde (K, FP64; +inf for non-finite), rho = min_k S_k, the normaliser
 * eta = sum_k exp(-(S_k - rho) / lambda), and the applied update dU (T x m FP64). */
int mppi_debug_last(mppi_ctx *ctx, double *costs, double *rho, double *eta, double *dU);

/* The standard normals the device draws for samples [k0, k0 + nk) at `iteration`
 * (nk x T x m FP32, host), from the same device code the rollouts use. */
int mppi_debug_normals(mppi_ctx *ctx, uint64_t iteration, int32_t k0, int32_t nk, float *eps);

/* Raw Philox4x32-10 blocks on `device`: out[4i..4i+3] = philox(counters[4i..4i+3], seed).
 * counters and out are host arrays of 4n uint32. */
int mppi_debug_philox(int32_t device, uint64_t seed, const uint32_t *counters, int32_t n, uint32_t *out);

/* The rollouts' lane-group primitives (aligned groups of `group` = 4, 16 or 32 lanes of a
 * 64-lane wave) on `device`, over n_waves (1..4096) full waves.  a and b are host arrays
 * of 64 n_waves floats; out (host, 6 floats per lane) receives, for lane t with j = t mod
 * group: the inclusive prefix sum of a over lanes 0..j of its group, the exclusive one,
 * a of the group's last lane, the group's sum of a (computed in FP64, returned in the
 * group's first lane; other lanes unspecified), and the composition, in lane order, of
 * the maps x -> a x + b of lanes 0..j as (slope, offset) (group <= 16; NaN for 32).
 * EINVAL on a bad group, size or pointer. */
int mppi_debug_lane_groups(int32_t device, int32_t group, const float *a, const float *b, int32_t n_waves,
                           float *out);

/* The launch configuration a context chose (host output).  rollout_mode bits name the
 * compiled rollout variant: MPPI_ROLLOUT_COST_TO_GO (prefix costs recorded), _CRASH (crash
 * indicator), _STEP_SPLIT (the lanes of a sample share its horizon), _DIAGONAL (A chol(Sigma)
 * and the likelihood-ratio matrix are diagonal, so only their diagonal products are formed),
 * _FUSED (two kernels per iteration: each rollout block also writes its samples' weighted
 * noise sums against its own minimum, and the finalize, one block per 4 sequence
 * components, rescales and merges them; update_blocks is then 0.  Chosen wherever
 * MPPI_KERNELS_FUSED is available, see mppi_config.kernels);
 * rollout_lanes is the lanes per sample (the learned dynamics: 4, sixteen samples per wave). */
enum { MPPI_ROLLOUT_COST_TO_GO = 1, MPPI_ROLLOUT_CRASH = 2, MPPI_ROLLOUT_STEP_SPLIT = 4,
       MPPI_ROLLOUT_DIAGONAL = 8, MPPI_ROLLOUT_FUSED = 16 };
typedef struct {
  int32_t rollout_lanes;
  int32_t rollout_mode;
  int32_t rollout_blocks;     /* rollout blocks per iteration                               */
  int32_t update_chunk;       /* samples per update block                                  */
  int32_t update_blocks;      /* update blocks per iteration                               */
  int32_t noise_groups;       /* Philox4x32-10 blocks per sample and iteration, ceil(T m/4) */
  uint64_t workspace_bytes;   /* device bytes of the context's state                       */
} mppi_info;
int mppi_get_info(mppi_ctx *ctx, mppi_info *out);

/* Kernel timing.  While profiling is on, every kernel of mppi_step / mppi_step_async is
 * launched directly (no graph) between two hipEvents recorded on the context's stream.
 * mppi_kernel_times waits for the stream and returns, per kernel kind (0 = rollout,
 * 1 = update, 2 = finalize), the mean duration in milliseconds and the number of
 * launches timed since profiling was switched on (avg_ms[3], count[3], host); a fused
 * context (MPPI_ROLLOUT_FUSED) launches no update, so its count stays 0. */
int mppi_set_profiling(mppi_ctx *ctx, int32_t on);
int mppi_kernel_times(mppi_ctx *ctx, double *avg_ms, int64_t *count);

/* ------------------------------------------------------------------------------------
 * Learned dynamics (extension of the model the paper samples from, Section II):
 * an MLP [16 -> 128 -> 128 -> 12] with tanh hidden layers maps the standardised
 * (state x[12], control u[4]) of the quadrotor to its standardised one-step state change;
 * MPPI_SYS_QUADROTOR_MLP rolls out x <- x + sd_out * MLP((z - mu_in) / sd_in) + mu_out.
 * All matrix products run on BF16 MFMA with FP32 accumulation: weights and activations are
 * rounded to bfloat16 (nearest even) at every product input, forward and backward.
 *
 * Parameters are one FP32 array of MPPI_MLP_PARAMS values in this order:
 *   W1 [128][16], b1 [128], W2 [128][128], b2 [128], W3 [12][128], b3 [12]   (row-major)
 * Statistics are one FP64 array of MPPI_MLP_STATS values: mu_in[16], sd_in[16],
 * mu_out[12], sd_out[12].
 * Training minimises the mean squared error of the standardised prediction with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 parameters; every kernel of the forward,
 * the backward and the optimiser is this library's own.
 * ------------------------------------------------------------------------------------ */
#define MPPI_MLP_PARAMS 20236
#define MPPI_MLP_STATS 56

/* Create a network on `device` from FP32 parameters (host, copied); statistics start as
 * mu = 0, sd = 1. */
int mppi_mlp_create(int32_t device, const float *params, mppi_mlp **out);
int mppi_mlp_destroy(mppi_mlp *mlp);
/* Training set: n >= 1 (state, control) pairs (host FP64, x: n x 12, u: n x 4, copied).  The
 * targets dx = dt f(x, u) are computed on the device with the analytic quadrotor model of
 * `quad`, and the standardisation statistics are set from the set (population mean and
 * standard deviation, FP64 sums on the device; a zero deviation is replaced by 1). */
int mppi_mlp_set_dataset(mppi_mlp *mlp, const mppi_quadrotor_params *quad, double dt, const double *x,
                         const double *u, int64_t n);
/* Read back the device-computed targets (n x 12 FP64). */
int mppi_mlp_get_targets(mppi_mlp *mlp, double *dx, int64_t n);
int mppi_mlp_set_stats(mppi_mlp *mlp, const double *stats);
int mppi_mlp_get_stats(mppi_mlp *mlp, double *stats);
int mppi_mlp_get_params(mppi_mlp *mlp, float *params);
int mppi_mlp_set_params(mppi_mlp *mlp, const float *params);
/* floor(n_order / batch) Adam steps; step s uses dataset rows order[s*batch .. (s+1)*batch)
 * (host int32, each in [0, n)).  losses (host, may be NULL) receives each step's loss
 * (mean squared error before the step).  1 <= batch <= 65536.  Blocks until done. */
int mppi_mlp_train(mppi_mlp *mlp, const int32_t *order, int64_t n_order, int32_t batch, double lr,
                   double *losses);
/* One forward + backward without an update on given standardised inputs zn (B x 16) and
 * targets tn (B x 12) (host FP64): the loss and the gradient (MPPI_MLP_PARAMS FP32, host). */
int mppi_mlp_loss_grads(mppi_mlp *mlp, const double *zn, const double *tn, int32_t B, double *loss, float *grads);
/* Predicted one-step change dx (B x 12) for states x (B x 12) and controls u (B x 4). */
int mppi_mlp_forward(mppi_mlp *mlp, const double *x, const double *u, int32_t B, double *dx);

/* ------------------------------------------------------------------------------------
 * Serving: many controllers on one GPU with continuous batching.
 *
 * Controllers are admitted into slots while their device state fits the HBM budget; their
 * warm-started sequences, iteration counters (which key the noise) and descriptors stay
 * resident on the device.  Each submitted request is one control step (one iteration,
 * emit u0, warm shift) of one controller from a given start state.  A controller has at
 * most one step in flight; its requests run in submission order.  Whenever one of the
 * server's streams is free, every controller with a pending request is packed into one
 * batch: one rollout launch per system present, one update launch and one finalize
 * launch cover all of them, so requests that arrive while other batches run join the
 * next batch and overlap with those on the device.  A controller's results are the same
 * alone and in any batch (the batched kernels run the single-controller code per block
 * and every reduction has a fixed order).  The real-time control loop of the paper runs
 * each controller at 50 Hz (Section V); the server reports per-request completion times.
 *
 * MPPI_SERVE_BATCHED_GRAPH forms the same batches but runs each as one graph launch: each
 * server stream keeps one instantiated graph per set of system types a batch can hold (the
 * plan upload, the types' rollouts as parallel branches, the update, the finalize and the
 * result download), and a launch only rewrites its kernel nodes' grid sizes and counts for
 * the batch at hand.  Its results are the same bit for bit; it is not the default because a
 * run at the scale of 256 controllers under a session trace ended the process with a host
 * segmentation fault whose cause has not been found.
 * MPPI_SERVE_PLAIN is the reference policy: one controller step at a time in arrival
 * order, each through the controller's own captured single-controller graph.
 * ------------------------------------------------------------------------------------ */
typedef struct mppi_server mppi_server;

enum { MPPI_SERVE_BATCHED = 0, MPPI_SERVE_PLAIN = 1, MPPI_SERVE_BATCHED_GRAPH = 2 };

typedef struct {
  int32_t device;
  uint64_t hbm_budget_bytes;  /* admission budget for controller device state              */
  int32_t max_slots;          /* 1 .. 4096 controllers                                     */
  int32_t max_inflight;       /* concurrent batches (one stream each), 1 .. 8; PLAIN uses 1 */
  int32_t max_batch;          /* controllers per batch, 1 .. max_slots                     */
  int32_t mode;               /* MPPI_SERVE_BATCHED, MPPI_SERVE_PLAIN or _BATCHED_GRAPH    */
} mppi_server_config;

typedef struct {
  uint64_t bytes_used;        /* device bytes held by admitted controllers                 */
  int32_t slots_used;
  int32_t queued;             /* requests waiting                                           */
  int32_t inflight;           /* requests on the device                                     */
  int64_t requests_done;
  int64_t batches;            /* batches launched                                           */
  double mean_batch;          /* requests per batch                                         */
  int64_t rollout_steps_done; /* sum of K * T over completed requests                       */
} mppi_server_stats;

int mppi_server_create(const mppi_server_config *cfg, mppi_server **out);
/* Drain everything in flight and free the server and all its controllers. */
int mppi_server_destroy(mppi_server *srv);
/* Admit a controller (cfg as for mppi_create; its stream and workspace fields are ignored).
 * MPPI_EBUSY when no slot is free or its device state would exceed the budget. */
int mppi_server_admit(mppi_server *srv, const mppi_config *cfg, int32_t *slot);
/* Free a slot and its device memory; MPPI_EBUSY while it has queued or in-flight steps. */
int mppi_server_release(mppi_server *srv, int32_t slot);
/* Queue one control step of `slot` from start state x0 (host, n doubles).  t_arrival is
 * on the server clock (mppi_server_now) and is only recorded. */
int mppi_server_submit(mppi_server *srv, int32_t slot, const double *x0, uint64_t req_id, double t_arrival);
/* Make progress (harvest finished batches, launch new ones) and return up to max finished
 * requests: req_ids[max], u0s[max x 4] (first m used), status[max] (MPPI_OK or
 * MPPI_ENUMERIC), t_done[max] on the server clock; *n = number written. */
int mppi_server_poll(mppi_server *srv, int32_t max, uint64_t *req_ids, double *u0s, int32_t *status,
                     double *t_done, int32_t *n);
/* Replay an arrival trace in real time: request i of slot slots[i] arrives t_arrival[i]
 * seconds after the call starts, from start state x0s[16 i .. 16 i + n); returns when all
 * are done, with t_done[i] (seconds since the start), u0s[4 i ..] and status[i].  Arrival
 * times must be non-decreasing. */
int mppi_server_replay(mppi_server *srv, int32_t n, const double *t_arrival, const int32_t *slots,
                       const double *x0s, double *t_done, double *u0s, int32_t *status);
/* Replay a trace of controller sessions with admission by the HBM budget: controllers that
 * arrive, wait for a slot and budget, run their 50 Hz loop (Section V) and leave.  Session j
 * (configuration cfgs[j], as for mppi_server_admit) arrives t_start[j] seconds after the call
 * starts and ends at t_end[j] >= t_start[j].  Arriving sessions wait in one first-come queue;
 * the head is admitted as soon as mppi_server_admit finds a slot and budget for it (the
 * sessions behind it wait too).  Request i of session sessions[i] arrives t_arrival[i], within
 * [t_start, t_end) of its session (non-decreasing over i), from x0s[16 i .. 16 i + n); it is
 * submitted when its session is admitted, so its latency includes any admission wait.  A
 * session is released once its end has passed (or the trace's last request has arrived) and
 * all its requests are served, which frees its slot and bytes for the queue.  Returns when
 * every request is done and every session has left, with t_done[i], u0s[4 i ..] and status[i]
 * per request (MPPI_EBUSY, not served, for a session whose state alone exceeds the budget)
 * and t_admit[j], t_release[j] per session (seconds since the start; -1 if never admitted).
 * Slots admitted before the call keep their share of the budget. */
int mppi_server_replay_sessions(mppi_server *srv, int32_t n_sessions, const mppi_config *cfgs,
                                const double *t_start, const double *t_end, int32_t n, const double *t_arrival,
                                const int32_t *sessions, const double *x0s, double *t_done, double *u0s,
                                int32_t *status, double *t_admit, double *t_release);
int mppi_server_stats_get(mppi_server *srv, mppi_server_stats *out);
/* Nominal sequence (T x m FP64) of an admitted controller, after its finished steps. */
int mppi_server_get_controls(mppi_server *srv, int32_t slot, double *u, uint64_t len);
/* Seconds on the server clock (steady, since creation). */
double mppi_server_now(mppi_server *srv);

/* Thread-local description of the last failure ("" if none). */
const char *mppi_last_error(void);

/* Library version string. */
const char *mppi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPPI_H */
