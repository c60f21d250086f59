// Host runtime and C ABI of libmppi (declarations and contracts: include/mppi.h).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mppi.h"
#include "mppi_kernels.h"
#include "mppi_runtime.h"

using namespace mppi;

// ----------------------------------------------------------------------- errors
namespace mppi {
thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(MPPI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace mppi

#define HIP_TRY(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return hip_fail(_e, #call);   \
  } while (0)

extern "C" const char *mppi_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *mppi_version(void) { return "libmppi 1.0 (gfx950)"; }

// ------------------------------------------------------------- config validation
namespace mppi {

static bool finite_all(const double *p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Lower Cholesky factor of an m x m SPD matrix (row-major); all-zero => zero factor.
static bool cholesky(const double *S, int m, double *L) {
  bool zero = true;
  for (int i = 0; i < m * m; ++i) zero = zero && S[i] == 0.0;
  for (int i = 0; i < m * m; ++i) L[i] = 0.0;
  if (zero) return true;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = S[i * m + j];
      for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i * m + i] = std::sqrt(s);
      } else {
        L[i * m + j] = s / L[j * m + j];
      }
    }
  return true;
}

static bool invert(const double *A, int m, double *Ai) {
  double a[16], b[16];
  for (int i = 0; i < m * m; ++i) { a[i] = A[i]; b[i] = 0.0; }
  for (int i = 0; i < m; ++i) b[i * m + i] = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(a[r * m + c]) > std::fabs(a[piv * m + c])) piv = r;
    if (a[piv * m + c] == 0.0) return false;
    for (int k = 0; k < m; ++k) { std::swap(a[c * m + k], a[piv * m + k]); std::swap(b[c * m + k], b[piv * m + k]); }
    const double d = a[c * m + c];
    for (int k = 0; k < m; ++k) { a[c * m + k] /= d; b[c * m + k] /= d; }
    for (int r = 0; r < m; ++r)
      if (r != c) {
        const double f = a[r * m + c];
        for (int k = 0; k < m; ++k) { a[r * m + k] -= f * a[c * m + k]; b[r * m + k] -= f * b[c * m + k]; }
      }
  }
  for (int i = 0; i < m * m; ++i) Ai[i] = b[i];
  return true;
}

static int expected_dims(int sys, int *n, int *m) {
  switch (sys) {
    case MPPI_SYS_LINEAR: return 0;  // checked separately
    case MPPI_SYS_CARTPOLE: *n = 4; *m = 1; return 1;
    case MPPI_SYS_CARTPOLE_SWINGUP: *n = 4; *m = 1; return 1;
    case MPPI_SYS_BICYCLE: *n = 5; *m = 2; return 1;
    case MPPI_SYS_QUADROTOR: *n = 12; *m = 4; return 1;
    case MPPI_SYS_QUADROTOR_MLP: *n = 12; *m = 4; return 1;
    default: return -1;
  }
}

int validate_config(const mppi_config *c) {
  if (!c) return fail(MPPI_EINVAL, "config is NULL");
  if (c->abi_version != MPPI_ABI_VERSION) return fail(MPPI_EINVAL, "abi_version %d != %d", c->abi_version, MPPI_ABI_VERSION);
  int n = 0, m = 0;
  const int d = expected_dims(c->system, &n, &m);
  if (d < 0) return fail(MPPI_EINVAL, "unknown system %d", c->system);
  if (d == 1 && (c->n_state != n || c->n_ctrl != m))
    return fail(MPPI_EINVAL, "system %d needs n_state=%d n_ctrl=%d (got %d, %d)", c->system, n, m, c->n_state, c->n_ctrl);
  if (c->system == MPPI_SYS_LINEAR) {
    if (c->n_state < 1 || c->n_state > 4) return fail(MPPI_EINVAL, "linear system: n_state must be in [1, 4]");
    if (c->n_ctrl != 1 && c->n_ctrl != 2 && c->n_ctrl != 4) return fail(MPPI_EINVAL, "linear system: n_ctrl must be 1, 2 or 4");
  }
  if (c->K < 1 || c->K > (1 << 22)) return fail(MPPI_EINVAL, "K=%d outside [1, 4194304]", c->K);
  if (c->T < 1 || c->T > 1024) return fail(MPPI_EINVAL, "T=%d outside [1, 1024]", c->T);
  if ((int64_t)c->T * c->n_ctrl > kMaxTM) return fail(MPPI_EINVAL, "T*n_ctrl exceeds %d", kMaxTM);
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return fail(MPPI_EINVAL, "dt must be finite and > 0");
  if (!(c->lambda > 0.0) || !std::isfinite(c->lambda)) return fail(MPPI_EINVAL, "lambda must be finite and > 0");
  if (!(c->nu > 0.0) || !std::isfinite(c->nu)) return fail(MPPI_EINVAL, "nu must be finite and > 0");
  if (!c->sigma) return fail(MPPI_EINVAL, "sigma is NULL");
  if (!c->u_init) return fail(MPPI_EINVAL, "u_init is NULL");
  if (!c->params) return fail(MPPI_EINVAL, "params is NULL");
  const int mm = c->n_ctrl;
  if (!finite_all(c->sigma, mm * mm)) return fail(MPPI_EINVAL, "sigma has non-finite entries");
  if (c->R && !finite_all(c->R, mm * mm)) return fail(MPPI_EINVAL, "R has non-finite entries");
  if (!finite_all(c->u_init, mm)) return fail(MPPI_EINVAL, "u_init has non-finite entries");
  if (c->nu_diag)
    for (int j = 0; j < mm; ++j)
      if (!(c->nu_diag[j] > 0.0) || !std::isfinite(c->nu_diag[j])) return fail(MPPI_EINVAL, "nu_diag entries must be finite and > 0");
  if (c->weighting != MPPI_WEIGHT_PATH && c->weighting != MPPI_WEIGHT_COST_TO_GO)
    return fail(MPPI_EINVAL, "unknown weighting %d", c->weighting);
  if (c->kernels != MPPI_KERNELS_AUTO && c->kernels != MPPI_KERNELS_FUSED && c->kernels != MPPI_KERNELS_THREE)
    return fail(MPPI_EINVAL, "unknown kernels value %d", c->kernels);
  if (c->kernels == MPPI_KERNELS_FUSED && !fused_available(c))
    return fail(MPPI_EINVAL, "the fused iteration needs at most %d rollout blocks and a block's normals within "
                "its LDS (%d bytes on the step-split systems, which under cost-to-go weighting also keep 32 KiB "
                "of running costs; the rest of %d on the quadrotor, under path weighting only)",
                kMaxMergedParts, kMaxFusedNormalsBytes, kMaxBlockLdsBytes);
  if (c->weighting == MPPI_WEIGHT_COST_TO_GO && c->system == MPPI_SYS_QUADROTOR_MLP)
    return fail(MPPI_EINVAL, "cost-to-go weighting is not available with the learned dynamics");
  if (c->u_nominal0 && !finite_all(c->u_nominal0, c->T * mm)) return fail(MPPI_EINVAL, "u_nominal0 has non-finite entries");
  for (int i = 0; i < mm; ++i)
    for (int j = 0; j < i; ++j)
      if (c->sigma[i * mm + j] != c->sigma[j * mm + i]) return fail(MPPI_EINVAL, "sigma is not symmetric");
  double L[16];
  if (!cholesky(c->sigma, mm, L)) return fail(MPPI_EINVAL, "sigma is not positive definite (or zero)");
  if (!c->R) {
    double Si[16];
    if (!invert(c->sigma, mm, Si)) return fail(MPPI_EINVAL, "R = NULL needs an invertible sigma");
  }
  size_t want = 0;
  switch (c->system) {
    case MPPI_SYS_LINEAR: want = sizeof(mppi_linear_params); break;
    case MPPI_SYS_CARTPOLE: want = sizeof(mppi_cartpole_params); break;
    case MPPI_SYS_CARTPOLE_SWINGUP: want = sizeof(mppi_swingup_params); break;
    case MPPI_SYS_BICYCLE: want = sizeof(mppi_bicycle_params); break;
    case MPPI_SYS_QUADROTOR: want = sizeof(mppi_quadrotor_params); break;
    case MPPI_SYS_QUADROTOR_MLP: want = sizeof(mppi_quadrotor_mlp_params); break;
  }
  if (c->params_bytes != want) return fail(MPPI_EINVAL, "params_bytes %llu != %zu for system %d",
                                           (unsigned long long)c->params_bytes, want, c->system);
  if (c->system == MPPI_SYS_LINEAR) {
    const auto *p = (const mppi_linear_params *)c->params;
    if (!p->A || !p->B || !p->Q || !p->Qf) return fail(MPPI_EINVAL, "linear params: NULL matrix");
  } else if (c->system == MPPI_SYS_CARTPOLE_SWINGUP) {
    const auto *p = (const mppi_swingup_params *)c->params;
    if (!(p->half_length > 0) || !std::isfinite(p->half_length) || !std::isfinite(p->gain) || !std::isfinite(p->gravity))
      return fail(MPPI_EINVAL, "swing-up params: half_length must be finite and > 0, gain and gravity finite");
  } else if (c->system == MPPI_SYS_BICYCLE) {
    const auto *p = (const mppi_bicycle_params *)c->params;
    if (!p->map || p->map_w < 2 || p->map_h < 2 || p->map_w > 16384 || p->map_h > 16384)
      return fail(MPPI_EINVAL, "bicycle params: need a map of at least 2 x 2 cells (at most 16384 per side)");
    if (!(p->cell_size > 0) || !(p->wheelbase > 0)) return fail(MPPI_EINVAL, "bicycle params: cell_size and wheelbase must be > 0");
  } else if (c->system == MPPI_SYS_QUADROTOR || c->system == MPPI_SYS_QUADROTOR_MLP) {
    const mppi_quadrotor_params *p = c->system == MPPI_SYS_QUADROTOR
                                         ? (const mppi_quadrotor_params *)c->params
                                         : &((const mppi_quadrotor_mlp_params *)c->params)->quad;
    if (p->n_obstacles < 0 || p->n_obstacles > QuadrotorSys::kMaxObstacles)
      return fail(MPPI_EINVAL, "quadrotor params: n_obstacles outside [0, %d]", QuadrotorSys::kMaxObstacles);
    if (p->n_obstacles > 0 && !p->obstacles) return fail(MPPI_EINVAL, "quadrotor params: obstacles is NULL");
    // finite spheres of radius + margin at most 1e6 and w_obs at most 1e12: the device obstacles
    // are scaled by a power of two s with s (r + margin)^2 <= 1/4, their weight by 1 / s^2,
    // which then stays finite in FP32
    if (!(p->obs_margin >= 0) || !std::isfinite(p->obs_margin) || !(p->w_obs >= 0) || !(p->w_obs <= 1e12) ||
        !std::isfinite(p->w_goal))
      return fail(MPPI_EINVAL, "quadrotor params: obs_margin must be finite and >= 0, w_obs in [0, 1e12], w_goal finite");
    for (int j = 0; j < p->n_obstacles; ++j) {
      const double *o = p->obstacles + 4 * j;
      if (!std::isfinite(o[0]) || !std::isfinite(o[1]) || !std::isfinite(o[2]) || !(o[3] >= 0) ||
          !(o[3] + p->obs_margin <= 1e6))
        return fail(MPPI_EINVAL, "quadrotor params: obstacle %d needs a finite centre and a radius in [0, 1e6 - margin]", j);
    }
    if (!(p->mass > 0) || !(p->inertia[0] > 0) || !(p->inertia[1] > 0) || !(p->inertia[2] > 0))
      return fail(MPPI_EINVAL, "quadrotor params: mass and inertia must be > 0");
    if (c->system == MPPI_SYS_QUADROTOR_MLP && !((const mppi_quadrotor_mlp_params *)c->params)->mlp)
      return fail(MPPI_EINVAL, "quadrotor_mlp params: mlp is NULL");
    if (!(p->crash_cost >= 0) || !std::isfinite(p->crash_cost) || !std::isfinite(p->ground_z))
      return fail(MPPI_EINVAL, "quadrotor params: crash_cost must be finite and >= 0, ground_z finite");
    if (c->system == MPPI_SYS_QUADROTOR_MLP && p->crash_cost != 0)
      return fail(MPPI_EINVAL, "the crash indicator is not available with the learned dynamics");
  }
  return MPPI_OK;
}

// ------------------------------------------------------------ workspace layout
static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// The step-split rollout serves the systems whose cost does not act on the state.
bool rollout_split(const mppi_config *c) {
  return c->system == MPPI_SYS_LINEAR || c->system == MPPI_SYS_CARTPOLE ||
         c->system == MPPI_SYS_CARTPOLE_SWINGUP || c->system == MPPI_SYS_BICYCLE;
}

// Lanes per sample of the rollout.  Step-split: 16 while K x 16 lanes stay within two
// waves per SIMD (K <= 8192), which trades redundant dynamics for a shorter chain per
// wave on a device the controller cannot fill; 4 for larger K, where the device is full
// and the redundancy would cost throughput.  The bicycle, whose chunk is all prefix
// scans (so a lane's chain shrinks with the group), takes 32 while K <= 4096: two waves
// per SIMD, each with half the chunks.  Otherwise the four-lane body's build value.
int rollout_lps(const mppi_config *c) {
  if (!rollout_split(c)) return MPPI_ROLLOUT_LPS;
  if (c->system == MPPI_SYS_BICYCLE && c->K <= 4096) return 32;
  return c->K <= 8192 ? 16 : 4;
}

// LDS floats of a four-lane (quadrotor) rollout block: controls, R u_i, u_i'R u_i / 2, the
// obstacles and (fused) the block's normals and weights.
static int64_t quad_rollout_lds_floats(const mppi_config *c, int n_obs, bool fused) {
  const int64_t T = c->T, m = c->n_ctrl, G = (T * m + 3) / 4, spb = kBlock / MPPI_ROLLOUT_LPS;
  int64_t fl = ((2 * T * m + ((T + 3) & ~3) + 3) & ~3) + (int64_t)QuadrotorSys::stage_floats(n_obs, 0);
  if (fused) fl = ((fl + 3) & ~3) + spb * (G * 4 + 2);
  return fl;
}

// Whether a step-split rollout block keeps its samples' running costs in LDS under cost-to-go
// weighting (at most 32 KiB of them), forming its own per-step minima.
static bool ctg_fold_fits(const mppi_config *c) {
  if (!rollout_split(c)) return false;
  return (int64_t)(kBlock / rollout_lps(c)) * (c->T + 1) * 8 <= 32768;
}

// The fused iteration, with every rollout block's partials mergeable by one finalize block: a
// step-split system whose rollout block's normals fit its LDS share (under cost-to-go
// weighting also its running costs), or the quadrotor under path weighting whose block's
// normals fit the rest of the CU's LDS.
bool fused_available(const mppi_config *c) {
  const int64_t G = ((int64_t)c->T * c->n_ctrl + 3) / 4;
  if (rollout_split(c)) {
    if (c->weighting != MPPI_WEIGHT_PATH && !ctg_fold_fits(c)) return false;
    const int spb = kBlock / rollout_lps(c);
    const int64_t n_roll = ((int64_t)c->K + spb - 1) / spb;
    return n_roll <= kMaxMergedParts && spb * G * 16 <= kMaxFusedNormalsBytes;
  }
  if (c->system != MPPI_SYS_QUADROTOR || c->weighting != MPPI_WEIGHT_PATH) return false;
  const auto *q = (const mppi_quadrotor_params *)c->params;
  const int spb = kBlock / MPPI_ROLLOUT_LPS;
  const int64_t n_roll = ((int64_t)c->K + spb - 1) / spb;
  return n_roll <= kMaxMergedParts &&
         4 * quad_rollout_lds_floats(c, q->n_obstacles, true) + 64 <= kMaxBlockLdsBytes;
}

// Whether MPPI_KERNELS_AUTO takes the fused iteration where it is available: always on the
// step-split systems; on the quadrotor while its rollout blocks number at most the MI355X's
// 256 CUs (K <= 16384).  Its blocks' normals fill a CU's LDS, one block per CU: past that
// count the three-kernel rollout, several blocks per CU, measured faster (K = 65536:
// 0.177 against 0.185 ms per control step; even at K = 32768; 5 % the other way at 16384).
static bool auto_fused(const mppi_config *c) {
  if (rollout_split(c)) return true;
  const int spb = kBlock / MPPI_ROLLOUT_LPS;
  return ((int64_t)c->K + spb - 1) / spb <= kQuadFusedAutoBlocks;
}

void compute_layout(const mppi_config *c, Layout *L) {
  const int K = c->K, T = c->T, m = c->n_ctrl;
  L->TM = T * m;
  L->G = (L->TM + 3) / 4;
  // samples per rollout block: 64 for the learned dynamics (16 per wave), 256 / lanes-per-sample otherwise
  const int roll_per_block = c->system == MPPI_SYS_QUADROTOR_MLP ? 64 : kBlock / rollout_lps(c);
  L->n_roll_blocks = (K + roll_per_block - 1) / roll_per_block;
  // update chunk: the smallest of 128, 256, 512 samples that keeps the update grid within
  // ~500 (128) or ~1200 (256) blocks: a shorter per-thread chain wins while the device has
  // room, fewer blocks win once it is full (512 with path weighting only)
  const int gblk = (L->G + kUpdGroups - 1) / kUpdGroups;
  const bool ctg_w = c->weighting == MPPI_WEIGHT_COST_TO_GO;
  if (((K + 127) / 128) * gblk <= 500) L->upd_chunk = 128;
  else if (ctg_w || ((K + 255) / 256) * gblk <= 1200) L->upd_chunk = 256;
  else L->upd_chunk = 512;
  L->n_kc = (K + L->upd_chunk - 1) / L->upd_chunk;
  L->fused = fused_available(c) && (c->kernels == MPPI_KERNELS_FUSED || (c->kernels == MPPI_KERNELS_AUTO && auto_fused(c)));
  // the multi-block finalize with the fused rollout (its P rollout partials are too many for
  // one block); the update's few chunk partials merge faster in one block
  L->multi = L->fused;
  L->n_fin_blocks = L->multi ? (L->TM + kFinOut - 1) / kFinOut : 1;
  const int n_parts = L->fused ? L->n_roll_blocks : L->n_kc;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { uint64_t r = o; o = align256(o + bytes); return r; };
  L->off_x0 = take(16 * sizeof(double));
  L->off_res = take(8 * sizeof(double));      // u0[4], flags (int[4]) packed after
  L->off_iter = take(sizeof(uint64_t));
  L->off_U64 = take((uint64_t)L->TM * 8);
  L->off_U32 = take((uint64_t)L->TM * 4);
  L->off_S = take((uint64_t)K * 8);
  L->off_blk_min = take((uint64_t)L->n_roll_blocks * 8);
  const bool ctg = c->weighting == MPPI_WEIGHT_COST_TO_GO;
  L->off_eta_part = take((uint64_t)n_parts * (ctg ? T : 1) * 8);
  L->off_part = take((uint64_t)n_parts * L->G * 4 * 8);
  L->off_shadow = L->multi ? take((uint64_t)L->TM * 8) : 0;
  L->off_basis = L->multi ? take((uint64_t)5 * 16 * 8) : 0;
  // cost-to-go on the step-split body: the rollout blocks form each step's minimum over their
  // samples from running costs kept in LDS (at most 32 KiB of them), the update reduces those
  L->ctg_fold = ctg_w && ctg_fold_fits(c);
  L->off_blk_tail = L->ctg_fold ? take((uint64_t)L->n_roll_blocks * T * 8) : 0;
  L->off_dbg = take((uint64_t)(2 + L->TM) * 8);
  L->off_pre = ctg && !L->fused ? take((uint64_t)T * K * 8) : 0;   // read by the update only
  L->off_rho_step = ctg ? take((uint64_t)T * 8) : 0;
  L->off_rho = take(sizeof(double));
  uint64_t sys_bytes = 0;
  if (c->system == MPPI_SYS_BICYCLE) {
    const auto *p = (const mppi_bicycle_params *)c->params;
    sys_bytes = (uint64_t)p->map_w * p->map_h * 4;
  } else if (c->system == MPPI_SYS_QUADROTOR || c->system == MPPI_SYS_QUADROTOR_MLP) {
    const mppi_quadrotor_params *p = c->system == MPPI_SYS_QUADROTOR
                                         ? (const mppi_quadrotor_params *)c->params
                                         : &((const mppi_quadrotor_mlp_params *)c->params)->quad;
    sys_bytes = (uint64_t)(p->n_obstacles > 0 ? p->n_obstacles : 1) * 20;   // float4 + r^2 each
  }
  L->off_sys = take(sys_bytes > 0 ? sys_bytes : 16);
  L->off_extra = o;
  L->extra_bytes = extra_workspace_bytes(c);
  L->total = align256(o + L->extra_bytes);
}

}  // namespace mppi

// ---------------------------------------------------------------------- context

extern "C" int mppi_workspace_bytes(const mppi_config *cfg, uint64_t *bytes) {
  int rc = validate_config(cfg);
  if (rc) return rc;
  if (!bytes) return fail(MPPI_EINVAL, "bytes is NULL");
  Layout L;
  compute_layout(cfg, &L);
  *bytes = L.total;
  return MPPI_OK;
}

namespace mppi {

// Fill the per-system device parameter blocks from the host description.
static int build_params(mppi_ctx *c) {
  const mppi_config &cfg = c->cfg;
  switch (cfg.system) {
    case MPPI_SYS_LINEAR: {
      const auto *p = (const mppi_linear_params *)cfg.params;
      const int n = cfg.n_state, m = cfg.n_ctrl;
      LinearParams lp;
      std::memset(&lp, 0, sizeof(lp));
      lp.n = n;
      for (int r = 0; r < n; ++r) {
        for (int k = 0; k < n; ++k) {
          lp.A[r * 4 + k] = (float)p->A[r * n + k];
          lp.Ad[r * 4 + k] = p->A[r * n + k];
          lp.Q[r * 4 + k] = (float)p->Q[r * n + k];
          lp.Qf[r * 4 + k] = (float)p->Qf[r * n + k];
        }
        for (int k = 0; k < m; ++k) {
          lp.B[r * m + k] = (float)p->B[r * m + k];
          lp.Bd[r * m + k] = p->B[r * m + k];
        }
      }
      c->linear = lp;
      break;
    }
    case MPPI_SYS_CARTPOLE: {
      const auto *p = (const mppi_cartpole_params *)cfg.params;
      CartPoleSys::Params cp;
      cp.mc = (float)p->mass_cart; cp.mp = (float)p->mass_pole; cp.l = (float)p->half_length; cp.g = (float)p->gravity;
      cp.dmc = p->mass_cart; cp.dmp = p->mass_pole; cp.dl = p->half_length; cp.dg = p->gravity;
      for (int i = 0; i < 4; ++i) { cp.qd[i] = (float)p->q_diag[i]; cp.qfd[i] = (float)p->qf_diag[i]; }
      c->cartpole = cp;
      break;
    }
    case MPPI_SYS_CARTPOLE_SWINGUP: {
      const auto *p = (const mppi_swingup_params *)cfg.params;
      SwingUpSys::Params sp;
      const double k = 3.0 / (4.0 * p->half_length);
      sp.gain = (float)p->gain; sp.k = (float)k; sp.g = (float)p->gravity;
      sp.dgain = p->gain; sp.dk = k; sp.dg = p->gravity;
      sp.wp = (float)p->w_pos; sp.wa = (float)p->w_angle; sp.wv = (float)p->w_vel; sp.wr = (float)p->w_rate;
      c->swingup = sp;
      break;
    }
    case MPPI_SYS_BICYCLE: {
      const auto *p = (const mppi_bicycle_params *)cfg.params;
      BicycleSys::Params bp;
      bp.L_inv = (float)(1.0 / p->wheelbase); bp.dL_inv = 1.0 / p->wheelbase;
      bp.vt = (float)p->v_target; bp.ws = (float)p->w_speed;
      bp.cell_inv = (float)(1.0 / p->cell_size);
      bp.lim = (float)p->steer_limit; bp.dlim = p->steer_limit;
      bp.W = p->map_w; bp.H = p->map_h;
      bp.map = (const float *)(c->base + c->L.off_sys);
      HIP_TRY(hipMemcpy((void *)bp.map, p->map, (size_t)p->map_w * p->map_h * 4, hipMemcpyHostToDevice));
      c->bicycle = bp;
      break;
    }
    case MPPI_SYS_QUADROTOR:
    case MPPI_SYS_QUADROTOR_MLP: {
      const mppi_quadrotor_params *p = cfg.system == MPPI_SYS_QUADROTOR
                                           ? (const mppi_quadrotor_params *)cfg.params
                                           : &((const mppi_quadrotor_mlp_params *)cfg.params)->quad;
      QuadrotorSys::Params qp;
      qp.m_inv = (float)(1.0 / p->mass); qp.dm_inv = 1.0 / p->mass;
      qp.g = (float)p->gravity; qp.dg = p->gravity;
      qp.arm = (float)p->arm; qp.darm = p->arm;
      qp.kap = (float)p->yaw_coef; qp.dkap = p->yaw_coef;
      for (int i = 0; i < 3; ++i) {
        qp.J[i] = (float)p->inertia[i]; qp.dJ[i] = p->inertia[i];
        qp.Jinv[i] = (float)(1.0 / p->inertia[i]); qp.dJinv[i] = 1.0 / p->inertia[i];
        qp.goal[i] = (float)p->goal[i];
      }
      qp.wg = (float)p->w_goal; qp.wo = (float)p->w_obs; qp.margin = (float)p->obs_margin;
      qp.n_obs = p->n_obstacles;
      qp.crash = (float)p->crash_cost; qp.ground = (float)p->ground_z;
      qp.dt_m_inv = (float)(cfg.dt / p->mass);
      qp.dt_g = (float)(cfg.dt * p->gravity);
      for (int i = 0; i < 3; ++i) qp.dt_Jinv[i] = (float)(cfg.dt / p->inertia[i]);
      qp.dt_rev = (float)(cfg.dt / (2.0 * M_PI));
      const int no = p->n_obstacles;
      // the obstacle scale: the largest power of two (at most 1) with s (r + margin)^2 <= 1/4
      double max_rr = 0.0;
      for (int j = 0; j < no; ++j) {
        const double rr = p->obstacles[4 * j + 3] + p->obs_margin;
        max_rr = std::fmax(max_rr, rr * rr);
      }
      double sc = 1.0;
      while (sc * max_rr > 0.25) sc *= 0.5;
      qp.obs_scale = (float)sc;
      qp.wo_s = (float)(p->w_obs / (sc * sc));
      qp.gq = (float)(p->w_goal / sc);
      double gg = 0.0;
      for (int i = 0; i < 3; ++i) {
        qp.glin[i] = (float)(-2.0 * p->w_goal * p->goal[i]);
        gg += p->goal[i] * p->goal[i];
      }
      qp.gconst = (float)(p->w_goal * gg);
      float ob[(QuadrotorSys::kMaxObstacles + 1) * 5];
      std::memset(ob, 0, sizeof(ob));
      for (int j = 0; j < no; ++j) {   // s (2 c, (r + margin)^2 - |c|^2), then s ((r + margin)^2 - r^2)
        const double *o = p->obstacles + 4 * j;
        const double rr = o[3] + p->obs_margin;
        ob[4 * j + 0] = (float)(sc * 2.0 * o[0]); ob[4 * j + 1] = (float)(sc * 2.0 * o[1]);
        ob[4 * j + 2] = (float)(sc * 2.0 * o[2]);
        ob[4 * j + 3] = (float)(sc * (rr * rr - (o[0] * o[0] + o[1] * o[1] + o[2] * o[2])));
        ob[4 * (size_t)no + j] = (float)(sc * (rr * rr - o[3] * o[3]));
      }
      qp.obs = (const float4 *)(c->base + c->L.off_sys);
      HIP_TRY(hipMemcpy((void *)qp.obs, ob, (size_t)(no > 0 ? no : 1) * 5 * 4, hipMemcpyHostToDevice));
      c->quad = qp;
      break;
    }
  }
  return MPPI_OK;
}

template <class Sys>
static size_t rollout_lds_bytes(const mppi_ctx *c) {
  const int T = c->cfg.T, m = c->cfg.n_ctrl;
  size_t fl = (size_t)2 * T * m + ((T + 3) & ~3);
  fl = (fl + 3) & ~size_t(3);
  // the step-split body stages nothing beyond the controls (fused: and the block's normals
  // and weights); the quadrotor its obstacles (fused: then the block's normals and weights)
  if constexpr (!Sys::kStepSplit) return (size_t)quad_rollout_lds_floats(&c->cfg, c->quad.n_obs, c->L.fused) * 4;
  else if (c->L.fused && c->L.ctg_fold)           // normals, running costs, path costs, step minima
    fl += (size_t)(kBlock / rollout_lps(&c->cfg)) * (c->L.G * 4 + (c->cfg.T + 1) * 2) + (size_t)c->cfg.T * 2;
  else if (c->L.fused) fl += (size_t)(kBlock / rollout_lps(&c->cfg)) * (c->L.G * 4 + 2);
  else if (c->L.ctg_fold) fl += (size_t)(kBlock / rollout_lps(&c->cfg)) * (c->cfg.T + 1) * 2;
  return fl * 4;
}

// The rollout variant a context runs: step-split where the system allows it, else the
// four-lane body; recording prefix costs under cost-to-go weighting, and with the
// quadrotor's crash indicator when its crash_cost is positive.
static_assert(MPPI_ROLLOUT_COST_TO_GO == kRecordPrefix && MPPI_ROLLOUT_CRASH == kCrashOn &&
                  MPPI_ROLLOUT_STEP_SPLIT == kStepSplit && MPPI_ROLLOUT_DIAGONAL == kDiagLR &&
                  MPPI_ROLLOUT_FUSED == kFused,
              "mppi_info.rollout_mode bits");
static int rollout_mode(const mppi_ctx *c) {
  int mode = c->cfg.weighting == MPPI_WEIGHT_COST_TO_GO ? kRecordPrefix : 0;
  const int m = c->cfg.n_ctrl;
  bool diag = true;                                 // the FP32 copies the kernels use
  for (int r = 0; r < m; ++r)
    for (int j = 0; j < m; ++j)
      if (r != j && ((float)c->Ls[r * m + j] != 0.f || (float)c->Mq[r * m + j] != 0.f)) diag = false;
  if (diag) mode |= kDiagLR;
  if (c->L.fused) mode |= kFused;
  if (rollout_split(&c->cfg)) return mode | kStepSplit;
  if (c->cfg.system == MPPI_SYS_QUADROTOR && c->quad.crash > 0.f) mode |= kCrashOn;
  return mode;
}

template <class Sys, int Mode>
static const void *rollout_fn() {
  if constexpr (Sys::kStepSplit) return nullptr;                     // these run step-split
  else if constexpr ((Mode & kCrashOn) != 0 && !Sys::kCrash) return nullptr;
  else return (const void *)rollout_kernel<Sys, Sys::kLPS, Mode>;
}

template <class Sys, int Mode>
static const void *rollout_split_fn(int lps) {
  if constexpr (Sys::kStepSplit) {
    if constexpr (Sys::kLanes32)
      if (lps == 32) return (const void *)rollout_kernel<Sys, 32, Mode>;
    if (lps == 16) return (const void *)rollout_kernel<Sys, 16, Mode>;
    if (lps == 4) return (const void *)rollout_kernel<Sys, 4, Mode>;
  }
  return nullptr;
}

// kDiagL: 0 or kDiagLR, the same for every variant the mode maps to
template <class Sys, int kDiagL>
static const void *rollout_fn_for_base(int mode, int lps) {
  if (mode == (kStepSplit | kDiagL)) return rollout_split_fn<Sys, kStepSplit | kDiagL>(lps);
  if (mode == (kStepSplit | kFused | kDiagL)) return rollout_split_fn<Sys, kStepSplit | kFused | kDiagL>(lps);
  if (mode == (kStepSplit | kRecordPrefix | kDiagL)) return rollout_split_fn<Sys, kStepSplit | kRecordPrefix | kDiagL>(lps);
  if (mode == (kStepSplit | kFused | kRecordPrefix | kDiagL))
    return rollout_split_fn<Sys, kStepSplit | kFused | kRecordPrefix | kDiagL>(lps);
  switch (mode) {
    case kDiagL: return rollout_fn<Sys, kDiagL>();
    case kFused | kDiagL: return rollout_fn<Sys, kFused | kDiagL>();
    case kRecordPrefix | kDiagL: return rollout_fn<Sys, kRecordPrefix | kDiagL>();
    case kCrashOn | kDiagL: return rollout_fn<Sys, kCrashOn | kDiagL>();
    case kCrashOn | kFused | kDiagL: return rollout_fn<Sys, kCrashOn | kFused | kDiagL>();
    case kRecordPrefix | kCrashOn | kDiagL: return rollout_fn<Sys, kRecordPrefix | kCrashOn | kDiagL>();
    default: return nullptr;
  }
}

template <class Sys>
static const void *rollout_fn_for(int mode, int lps) {
  if (mode & kDiagLR) return rollout_fn_for_base<Sys, kDiagLR>(mode, lps);
  return rollout_fn_for_base<Sys, 0>(mode, lps);
}

static hipEvent_t take_event(mppi_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch fn on s. In profiling mode the start and stop events are taken by the launch
// itself, so the interval they bound holds this kernel alone (kind: 0 rollout).
int timed_launch(mppi_ctx *c, int kind, const void *fn, dim3 grid, dim3 block, void **args, size_t lds,
                 hipStream_t s) {
  hipEvent_t e0 = c->profiling ? take_event(c) : nullptr;
  hipEvent_t e1 = e0 ? take_event(c) : nullptr;
  if (e0 && !e1) { c->event_pool.push_back(e0); e0 = nullptr; }
  HIP_TRY(hipExtLaunchKernel(fn, grid, block, args, lds, s, e0, e1, 0));
  if (e0) c->pending.push_back({kind, e0, e1});
  return MPPI_OK;
}

template <class Sys>
static int launch_rollout(mppi_ctx *c, const IterArgs &a, const typename Sys::Params &p, hipStream_t s) {
  const size_t lds = rollout_lds_bytes<Sys>(c);
  const void *fn = rollout_fn_for<Sys>(rollout_mode(c), rollout_lps(&c->cfg));
  if (!fn) return fail(MPPI_EINVAL, "rollout variant not available for system %d", c->cfg.system);
  void *args[] = {(void *)&a, (void *)&p};
  const int extra = c->L.multi ? 1 : 0;              // the shadow / plant-basis block
  return timed_launch(c, 0, fn, dim3(c->L.n_roll_blocks + extra), dim3(kBlock), args, lds, s);
}

template <class Sys>
static int prepare_rollout(mppi_ctx *c) {
  const size_t lds = rollout_lds_bytes<Sys>(c);
  if (lds > 160 * 1024 - 64) return fail(MPPI_EINVAL, "rollout needs %zu B of LDS (T too large)", lds);
  const void *fn = rollout_fn_for<Sys>(rollout_mode(c), rollout_lps(&c->cfg));
  if (!fn) return fail(MPPI_EINVAL, "rollout variant not available for system %d", c->cfg.system);
  HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return MPPI_OK;
}

static IterArgs make_iter_args(mppi_ctx *c, const double *x0) {
  IterArgs a;
  std::memset(&a, 0, sizeof(a));
  const Layout &L = c->L;
  a.x0 = x0;
  a.U64 = (const double *)(c->base + L.off_U64);
  if (L.multi) a.Ushadow = (double *)(c->base + L.off_shadow);
  a.U32 = (const float *)(c->base + L.off_U32);
  a.S = (double *)(c->base + L.off_S);
  a.blk_min = (double *)(c->base + L.off_blk_min);
  a.iter = (const uint64_t *)(c->base + L.off_iter);
  a.part = (double *)(c->base + L.off_part);
  a.eta_part = (double *)(c->base + L.off_eta_part);
  if (c->cfg.weighting == MPPI_WEIGHT_COST_TO_GO) {
    if (!L.fused) a.pre = (double *)(c->base + L.off_pre);
    a.rho_step = (double *)(c->base + L.off_rho_step);
    if (L.ctg_fold) a.blk_tail = (double *)(c->base + L.off_blk_tail);
  }
  a.key0 = (uint32_t)c->cfg.seed;
  a.key1 = (uint32_t)(c->cfg.seed >> 32);
  a.n = c->cfg.n_state;
  a.K = c->cfg.K; a.T = c->cfg.T; a.m = c->cfg.n_ctrl; a.G = L.G;
  a.n_roll_blocks = L.n_roll_blocks; a.n_kc = L.n_kc;
  a.dt = (float)c->cfg.dt;
  const int m = c->cfg.n_ctrl;
  for (int i = 0; i < m * m; ++i) { a.Ls[i] = (float)c->Ls[i]; a.R[i] = (float)c->R[i]; a.Mq[i] = (float)c->Mq[i]; }
  a.inv_lambda = 1.0 / c->cfg.lambda;
  a.rho_out = (double *)(c->base + L.off_rho);
  a.upd_chunk = L.upd_chunk;
  return a;
}

static FinalizeArgs make_fin_args(mppi_ctx *c, double *u0_out, int emit) {
  FinalizeArgs f;
  std::memset(&f, 0, sizeof(f));
  const Layout &L = c->L;
  f.U64 = (double *)(c->base + L.off_U64);
  f.U32 = (float *)(c->base + L.off_U32);
  // the minimum: the update's (path weighting), or the first step's cost-to-go minimum,
  // which is the minimum path cost since no cost precedes step 0
  f.rho = c->cfg.weighting == MPPI_WEIGHT_COST_TO_GO ? (const double *)(c->base + L.off_rho_step)
                                                     : (const double *)(c->base + L.off_rho);
  f.part = (const double *)(c->base + L.off_part);
  f.eta_part = (const double *)(c->base + L.off_eta_part);
  f.iter = (uint64_t *)(c->base + L.off_iter);
  f.flags = (int *)(c->base + L.off_res + 4 * sizeof(double));
  f.dbg = (double *)(c->base + L.off_dbg);
  f.u0_out = u0_out;
  f.T = c->cfg.T; f.m = c->cfg.n_ctrl; f.G = L.G; f.n_kc = L.n_kc;
  f.emit = emit;
  f.ctg = c->cfg.weighting == MPPI_WEIGHT_COST_TO_GO;
  if (L.multi) {
    f.multi = 1;
    f.n_parts = L.n_roll_blocks;
    f.blk_min = (const double *)(c->base + L.off_blk_min);
    f.Ushadow = (const double *)(c->base + L.off_shadow);
    if (f.ctg) {
      f.blk_tail = (const double *)(c->base + L.off_blk_tail);
      f.rho_step = (double *)(c->base + L.off_rho_step);
    }
  }
  f.inv_lambda = 1.0 / c->cfg.lambda;
  for (int i = 0; i < 16; ++i) f.Ls[i] = c->Ls[i];
  for (int j = 0; j < c->cfg.n_ctrl; ++j) f.u_init[j] = c->u_init[j];
  return f;
}

// Record the start event of a timed kernel (profiling mode only).
static hipEvent_t prof_begin(mppi_ctx *c, hipStream_t s) {
  if (!c->profiling) return nullptr;
  hipEvent_t e = take_event(c);
  if (e) (void)hipEventRecord(e, s);
  return e;
}

static void prof_end(mppi_ctx *c, hipStream_t s, int kind, hipEvent_t start) {
  if (!c->profiling || !start) return;
  hipEvent_t e = take_event(c);
  if (!e) return;
  (void)hipEventRecord(e, s);
  c->pending.push_back({kind, start, e});
}

// Enqueue n_iters iterations (+ emit/shift) on stream s.
template <class Sys>
static void launch_finalize_plant(mppi_ctx *c, const FinalizeArgs &f, double *x, const typename Sys::Params &p,
                                  hipStream_t s) {
  if (c->L.multi)
    hipLaunchKernelGGL(finalize_multi_plant_kernel<Sys>, dim3(c->L.n_fin_blocks), dim3(kFinMultiBlock), 0, s, f, x,
                       c->cfg.dt, c->cfg.n_state, (const double *)(c->base + c->L.off_basis));
  else
    hipLaunchKernelGGL(finalize_plant_kernel<Sys>, dim3(1), dim3(kFinBlock), 0, s, f, x, c->cfg.dt, c->cfg.n_state, p);
}

// Last finalize of a step with the plant step fused (plant_x != NULL).
static void launch_finalize(mppi_ctx *c, const FinalizeArgs &f, double *plant_x, hipStream_t s) {
  if (!plant_x) {
    if (c->L.multi) hipLaunchKernelGGL(finalize_multi_kernel, dim3(c->L.n_fin_blocks), dim3(kFinMultiBlock), 0, s, f);
    else hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinBlock), 0, s, f);
    return;
  }
  switch (c->cfg.system) {
    case MPPI_SYS_LINEAR:
      if (c->cfg.n_ctrl == 1) launch_finalize_plant<LinearSys<1>>(c, f, plant_x, c->linear, s);
      else if (c->cfg.n_ctrl == 2) launch_finalize_plant<LinearSys<2>>(c, f, plant_x, c->linear, s);
      else launch_finalize_plant<LinearSys<4>>(c, f, plant_x, c->linear, s);
      break;
    case MPPI_SYS_CARTPOLE: launch_finalize_plant<CartPoleSys>(c, f, plant_x, c->cartpole, s); break;
    case MPPI_SYS_CARTPOLE_SWINGUP: launch_finalize_plant<SwingUpSys>(c, f, plant_x, c->swingup, s); break;
    case MPPI_SYS_BICYCLE: launch_finalize_plant<BicycleSys>(c, f, plant_x, c->bicycle, s); break;
    default: launch_finalize_plant<QuadrotorSys>(c, f, plant_x, c->quad, s); break;
  }
}

int enqueue_iterations(mppi_ctx *c, const double *x0_dev, int n_iters, double *u0_dev, hipStream_t s,
                       double *plant_x) {
  const IterArgs a0 = make_iter_args(c, x0_dev);
  for (int it = 0; it < n_iters; ++it) {
    int rc = MPPI_OK;
    IterArgs a = a0;
    if (c->L.multi && plant_x && it == n_iters - 1) {   // the rollout evaluates the plant basis
      a.plant_basis = (double *)(c->base + c->L.off_basis);
      a.plant_x = plant_x;
    }
    switch (c->cfg.system) {
      case MPPI_SYS_LINEAR:
        if (c->cfg.n_ctrl == 1) rc = launch_rollout<LinearSys<1>>(c, a, c->linear_as<1>(), s);
        else if (c->cfg.n_ctrl == 2) rc = launch_rollout<LinearSys<2>>(c, a, c->linear_as<2>(), s);
        else rc = launch_rollout<LinearSys<4>>(c, a, c->linear_as<4>(), s);
        break;
      case MPPI_SYS_CARTPOLE: rc = launch_rollout<CartPoleSys>(c, a, c->cartpole, s); break;
      case MPPI_SYS_CARTPOLE_SWINGUP: rc = launch_rollout<SwingUpSys>(c, a, c->swingup, s); break;
      case MPPI_SYS_BICYCLE: rc = launch_rollout<BicycleSys>(c, a, c->bicycle, s); break;
      case MPPI_SYS_QUADROTOR: rc = launch_rollout<QuadrotorSys>(c, a, c->quad, s); break;
      case MPPI_SYS_QUADROTOR_MLP: rc = launch_mlp_rollout(c, a, s); break;
    }
    if (rc) return rc;
    const dim3 ugrid(c->L.n_kc, (c->L.G + kUpdGroups - 1) / kUpdGroups);
    hipEvent_t t0 = nullptr;
    if (!c->L.fused) {                              // fused: the rollout wrote the partials
      t0 = prof_begin(c, s);
      if (a.pre) {
        if (!a.blk_tail) hipLaunchKernelGGL(stepmin_kernel, dim3(c->cfg.T), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(update_ctg_kernel, ugrid, dim3(kBlock), 0, s, a);
      } else {
        hipLaunchKernelGGL(update_kernel, ugrid, dim3(kBlock), 0, s, a);
      }
      prof_end(c, s, 1, t0);
    }
    const FinalizeArgs f = make_fin_args(c, u0_dev, it == n_iters - 1);
    t0 = prof_begin(c, s);
    launch_finalize(c, f, it == n_iters - 1 ? plant_x : nullptr, s);
    prof_end(c, s, 2, t0);
  }
  HIP_TRY(hipGetLastError());
  return MPPI_OK;
}

// Run n_iters iterations, through a cached hipGraph when enabled.
constexpr size_t kMaxGraphs = 16;   // captured step graphs kept per context

// n_steps control steps (closed loop: n_steps > 1 needs plant_x, and step j emits into
// u0_dev + j m), through a cached hipGraph when enabled.
static int enqueue_steps(mppi_ctx *c, const double *x0_dev, int n_iters, double *u0_dev, hipStream_t s,
                         double *plant_x, int n_steps) {
  for (int j = 0; j < n_steps; ++j) {
    const int rc = enqueue_iterations(c, x0_dev, n_iters, u0_dev + (size_t)j * c->cfg.n_ctrl, s, plant_x);
    if (rc) return rc;
  }
  return MPPI_OK;
}

int run_iterations(mppi_ctx *c, const double *x0_dev, int n_iters, double *u0_dev, double *plant_x, int n_steps) {
  if (!c->cfg.use_graph || c->profiling) return enqueue_steps(c, x0_dev, n_iters, u0_dev, c->stream, plant_x, n_steps);
  auto key = std::make_tuple(n_steps, n_iters, (const void *)x0_dev, (const void *)u0_dev, (const void *)plant_x);
  auto itg = c->graphs.find(key);
  if (itg == c->graphs.end()) {
    if (c->graphs.size() >= kMaxGraphs) {           // bounded cache: start over (none in flight)
      HIP_TRY(hipStreamSynchronize(c->stream));
      for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
      c->graphs.clear();
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t ge;
    // the capture stream is made on the first capture: contexts that never replay their own
    // graphs (the batched server's) hold none
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_steps(c, x0_dev, n_iters, u0_dev, c->cap_stream, plant_x, n_steps);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    itg = c->graphs.emplace(key, ge).first;
  }
  HIP_TRY(hipGraphLaunch(itg->second, c->stream));
  return MPPI_OK;
}

size_t ctx_rollout_lds(const mppi_ctx *c) {
  switch (c->cfg.system) {
    case MPPI_SYS_LINEAR: return rollout_lds_bytes<LinearSys<1>>(c);
    case MPPI_SYS_CARTPOLE: return rollout_lds_bytes<CartPoleSys>(c);
    case MPPI_SYS_CARTPOLE_SWINGUP: return rollout_lds_bytes<SwingUpSys>(c);
    case MPPI_SYS_BICYCLE: return rollout_lds_bytes<BicycleSys>(c);
    default: return rollout_lds_bytes<QuadrotorSys>(c);
  }
}

// Descriptor of a controller for the batched serving kernels (x0 / u0 come per batch).
void fill_desc(mppi_ctx *c, CtrlDesc *d) {
  std::memset(d, 0, sizeof(*d));
  d->it = make_iter_args(c, nullptr);
  d->fin = make_fin_args(c, nullptr, 1);
  switch (c->cfg.system) {
    case MPPI_SYS_LINEAR: d->p.lin = c->linear; break;
    case MPPI_SYS_CARTPOLE: d->p.cp = c->cartpole; break;
    case MPPI_SYS_CARTPOLE_SWINGUP: d->p.su = c->swingup; break;
    case MPPI_SYS_BICYCLE: d->p.bc = c->bicycle; break;
    default: d->p.qd = c->quad; break;
  }
}

int set_device(int dev) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(MPPI_EDEVICE, "no HIP device available");
  if (dev < 0 || dev >= n) return fail(MPPI_EINVAL, "device %d outside [0, %d)", dev, n);
  HIP_TRY(hipSetDevice(dev));
  return MPPI_OK;
}

}  // namespace mppi

namespace mppi {

// The host-side state of a context: the configuration, A chol(Sigma), R, the likelihood-ratio
// matrix (R - A^-1 R A^-1) / 2, u_init and the workspace layout (no device work).
static void init_host_state(mppi_ctx *c, const mppi_config *cfg) {
  c->cfg = *cfg;
  const int m = cfg->n_ctrl;
  cholesky(cfg->sigma, m, c->L64);
  // covariance change A = diag(sqrt(nu_j)) (sqrt(nu) I without per-dimension factors)
  double sq[4];
  for (int j = 0; j < m; ++j) sq[j] = std::sqrt(cfg->nu_diag ? cfg->nu_diag[j] : cfg->nu);
  for (int i = 0; i < 16; ++i) c->Ls[i] = 0.0;
  for (int r = 0; r < m; ++r)
    for (int l = 0; l < m; ++l) c->Ls[r * m + l] = sq[r] * c->L64[r * m + l];
  if (cfg->R) {
    for (int i = 0; i < m * m; ++i) c->R[i] = cfg->R[i];
  } else {
    double Si[16];
    invert(cfg->sigma, m, Si);
    for (int i = 0; i < m * m; ++i) c->R[i] = cfg->lambda * Si[i];
  }
  for (int r = 0; r < m; ++r)
    for (int l = 0; l < m; ++l) c->Mq[r * m + l] = 0.5 * c->R[r * m + l] * (1.0 - 1.0 / (sq[r] * sq[l]));
  for (int j = 0; j < m; ++j) c->u_init[j] = cfg->u_init[j];
  c->cfg.sigma = c->cfg.R = c->cfg.u_init = c->cfg.u_nominal0 = c->cfg.nu_diag = nullptr;  // not kept
  compute_layout(cfg, &c->L);
}

// Per-system preparation of the rollout kernel (dynamic LDS size) once buffers are placed.
static int prepare_system(mppi_ctx *c) {
  const int m = c->cfg.n_ctrl;
  switch (c->cfg.system) {
    case MPPI_SYS_LINEAR:
      return m == 1 ? prepare_rollout<LinearSys<1>>(c) : (m == 2 ? prepare_rollout<LinearSys<2>>(c) : prepare_rollout<LinearSys<4>>(c));
    case MPPI_SYS_CARTPOLE: return prepare_rollout<CartPoleSys>(c);
    case MPPI_SYS_CARTPOLE_SWINGUP: return prepare_rollout<SwingUpSys>(c);
    case MPPI_SYS_BICYCLE: return prepare_rollout<BicycleSys>(c);
    case MPPI_SYS_QUADROTOR: return prepare_rollout<QuadrotorSys>(c);
    case MPPI_SYS_QUADROTOR_MLP: return prepare_mlp_rollout(c);
    default: return MPPI_OK;
  }
}

}  // namespace mppi

extern "C" int mppi_create(const mppi_config *cfg, mppi_ctx **out) {
  if (!out) return fail(MPPI_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_config(cfg);
  if (rc) return rc;
  rc = set_device(cfg->device);
  if (rc) return rc;
  auto *c = new mppi_ctx();
  init_host_state(c, cfg);
  const int m = cfg->n_ctrl, T = cfg->T;
  // device memory
  if (cfg->workspace) {
    if (cfg->workspace_bytes < c->L.total) {
      delete c;
      return fail(MPPI_ENOMEM, "workspace of %llu B < %llu B needed", (unsigned long long)cfg->workspace_bytes,
                  (unsigned long long)c->L.total);
    }
    if (((uintptr_t)cfg->workspace & 255) != 0) {
      delete c;
      return fail(MPPI_EINVAL, "workspace must be 256-byte aligned");
    }
    c->base = (char *)cfg->workspace;
    c->owns_ws = false;
  } else {
    hipError_t e = hipMalloc((void **)&c->base, c->L.total);
    if (e != hipSuccess) { delete c; return fail(MPPI_ENOMEM, "hipMalloc(%llu): %s", (unsigned long long)c->L.total, hipGetErrorString(e)); }
    c->owns_ws = true;
  }
  if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
    c->owns_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { mppi_destroy(c); return fail(MPPI_EDEVICE, "stream create failed"); }
    c->owns_stream = true;
  }
  if (hipHostMalloc((void **)&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) { mppi_destroy(c); return fail(MPPI_ENOMEM, "hipHostMalloc failed"); }
  rc = build_params(c);
  if (!rc) rc = init_extra(c, cfg);
  if (!rc) rc = prepare_system(c);
  if (rc) { std::string msg = g_last_error; mppi_destroy(c); g_last_error = msg; return rc; }
  // initial state: U (FP64 + FP32), iteration 0, zero flags
  std::vector<double> U((size_t)T * m);
  for (int i = 0; i < T; ++i)
    for (int j = 0; j < m; ++j) U[(size_t)i * m + j] = cfg->u_nominal0 ? cfg->u_nominal0[(size_t)i * m + j] : cfg->u_init[j];
  std::vector<float> U32(U.begin(), U.end());
  std::vector<char> zeros(c->L.off_U64, 0);
  hipError_t e = hipMemcpy(c->base, zeros.data(), zeros.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->base + c->L.off_U64, U.data(), U.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->base + c->L.off_U32, U32.data(), U32.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) { mppi_destroy(c); return hip_fail(e, "initial upload"); }
  *out = c;
  return MPPI_OK;
}

extern "C" int mppi_destroy(mppi_ctx *c) {
  if (!c) return MPPI_OK;
  (void)hipSetDevice(c->cfg.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto &t : c->pending) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  destroy_extra(c);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->owns_stream && c->stream) (void)hipStreamDestroy(c->stream);
  if (c->owns_ws && c->base) (void)hipFree(c->base);
  delete c;
  return MPPI_OK;
}

static int check_ctx(mppi_ctx *c) {
  if (!c) return fail(MPPI_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->cfg.device));
  return MPPI_OK;
}

static int collect_flags(mppi_ctx *c, int count) {
  if (count != c->seen_numeric) {
    c->seen_numeric = count;
    return fail(MPPI_ENUMERIC, "an iteration had no sample with a finite path cost; U was left unchanged");
  }
  return MPPI_OK;
}

extern "C" int mppi_step(mppi_ctx *c, const double *x0, int32_t n_iters, double *u0) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!x0 || !u0) return fail(MPPI_EINVAL, "x0 and u0 must be non-NULL");
  if (n_iters < 1 || n_iters > 1000) return fail(MPPI_EINVAL, "n_iters=%d outside [1, 1000]", n_iters);
  if (!finite_all(x0, c->cfg.n_state)) return fail(MPPI_EINVAL, "x0 has non-finite entries");
  double *px = (double *)c->pinned;
  const int n = c->cfg.n_state, m = c->cfg.n_ctrl;
  std::memcpy(px, x0, n * sizeof(double));
  double *d_x0 = (double *)(c->base + c->L.off_x0);
  double *d_res = (double *)(c->base + c->L.off_res);
  HIP_TRY(hipMemcpyAsync(d_x0, px, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  rc = run_iterations(c, d_x0, n_iters, d_res, nullptr);
  if (rc) return rc;
  char *pres = c->pinned + 1024;
  HIP_TRY(hipMemcpyAsync(pres, d_res, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(u0, pres, m * sizeof(double));
  int count;
  std::memcpy(&count, pres + 4 * sizeof(double), sizeof(int));
  return collect_flags(c, count);
}

extern "C" int mppi_step_async(mppi_ctx *c, const double *x0_dev, int32_t n_iters, double *u0_dev) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!x0_dev || !u0_dev) return fail(MPPI_EINVAL, "x0_dev and u0_dev must be non-NULL");
  if (n_iters < 1 || n_iters > 1000) return fail(MPPI_EINVAL, "n_iters=%d outside [1, 1000]", n_iters);
  return run_iterations(c, x0_dev, n_iters, u0_dev, nullptr);
}

extern "C" int mppi_step_plant_async(mppi_ctx *c, double *x_dev, int32_t n_iters, double *u0_dev) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!x_dev || !u0_dev) return fail(MPPI_EINVAL, "x_dev and u0_dev must be non-NULL");
  if (n_iters < 1 || n_iters > 1000) return fail(MPPI_EINVAL, "n_iters=%d outside [1, 1000]", n_iters);
  return run_iterations(c, x_dev, n_iters, u0_dev, x_dev);
}

extern "C" int mppi_run_closed_loop_async(mppi_ctx *c, double *x_dev, int32_t n_steps, int32_t n_iters,
                                          double *u_log_dev) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!x_dev || !u_log_dev) return fail(MPPI_EINVAL, "x_dev and u_log_dev must be non-NULL");
  if (n_steps < 1 || n_steps > 1000) return fail(MPPI_EINVAL, "n_steps=%d outside [1, 1000]", n_steps);
  if (n_iters < 1 || n_iters > 1000) return fail(MPPI_EINVAL, "n_iters=%d outside [1, 1000]", n_iters);
  if ((int64_t)n_steps * n_iters > 1000) return fail(MPPI_EINVAL, "n_steps * n_iters exceeds 1000");
  return run_iterations(c, x_dev, n_iters, u_log_dev, x_dev, n_steps);
}

extern "C" int mppi_sync(mppi_ctx *c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  char *pres = c->pinned + 2048;
  HIP_TRY(hipMemcpyAsync(pres, c->base + c->L.off_res + 4 * sizeof(double), sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  int count;
  std::memcpy(&count, pres, sizeof(int));
  return collect_flags(c, count);
}

extern "C" int mppi_plant_step_async(mppi_ctx *c, double *x_dev, const double *u_dev) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!x_dev || !u_dev) return fail(MPPI_EINVAL, "x_dev and u_dev must be non-NULL");
  const double dt = c->cfg.dt;
  switch (c->cfg.system) {
    case MPPI_SYS_LINEAR:
      if (c->cfg.n_ctrl == 1) hipLaunchKernelGGL(plant_kernel<LinearSys<1>>, dim3(1), dim3(64), 0, c->stream, x_dev, u_dev, dt, c->cfg.n_state, c->linear_as<1>());
      else if (c->cfg.n_ctrl == 2) hipLaunchKernelGGL(plant_kernel<LinearSys<2>>, dim3(1), dim3(64), 0, c->stream, x_dev, u_dev, dt, c->cfg.n_state, c->linear_as<2>());
      else hipLaunchKernelGGL(plant_kernel<LinearSys<4>>, dim3(1), dim3(64), 0, c->stream, x_dev, u_dev, dt, c->cfg.n_state, c->linear_as<4>());
      break;
    case MPPI_SYS_CARTPOLE: hipLaunchKernelGGL(plant_kernel<CartPoleSys>, dim3(1), dim3(64), 0, c->stream, x_dev, u_dev, dt, c->cfg.n_state, c->cartpole); break;
    case MPPI_SYS_CARTPOLE_SWINGUP: hipLaunchKernelGGL(plant_kernel<SwingUpSys>, dim3(1), dim3(64), 0, c->stream, x_dev, u_dev, dt, c->cfg.n_state, c->swingup); break;
    case MPPI_SYS_BICYCLE: hipLaunchKernelGGL(plant_kernel<BicycleSys>, dim3(1), dim3(64), 0, c->stream, x_dev, u_dev, dt, c->cfg.n_state, c->bicycle); break;
    case MPPI_SYS_QUADROTOR:
    case MPPI_SYS_QUADROTOR_MLP:
      hipLaunchKernelGGL(plant_kernel<QuadrotorSys>, dim3(1), dim3(64), 0, c->stream, x_dev, u_dev, dt, c->cfg.n_state, c->quad); break;
  }
  HIP_TRY(hipGetLastError());
  return MPPI_OK;
}

extern "C" int mppi_get_controls(mppi_ctx *c, double *u, uint64_t len) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!u || len != (uint64_t)c->L.TM) return fail(MPPI_EINVAL, "u must hold T*n_ctrl = %d doubles", c->L.TM);
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(u, c->base + c->L.off_U64, (size_t)c->L.TM * 8, hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" int mppi_set_controls(mppi_ctx *c, const double *u, uint64_t len) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!u || len != (uint64_t)c->L.TM) return fail(MPPI_EINVAL, "u must hold T*n_ctrl = %d doubles", c->L.TM);
  if (!finite_all(u, c->L.TM)) return fail(MPPI_EINVAL, "u has non-finite entries");
  std::vector<float> f(u, u + c->L.TM);
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(c->base + c->L.off_U64, u, (size_t)c->L.TM * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->base + c->L.off_U32, f.data(), (size_t)c->L.TM * 4, hipMemcpyHostToDevice));
  return MPPI_OK;
}

// State blob: magic, T*m, iteration, U64[T*m].
extern "C" int mppi_get_state(mppi_ctx *c, void *buf, uint64_t len, uint64_t *needed) {
  int rc = check_ctx(c);
  if (rc) return rc;
  const uint64_t need = 3 * 8 + (uint64_t)c->L.TM * 8;
  if (needed) *needed = need;
  if (!buf) return MPPI_OK;
  if (len < need) return fail(MPPI_EINVAL, "state buffer of %llu B < %llu B", (unsigned long long)len, (unsigned long long)need);
  uint64_t *h = (uint64_t *)buf;
  h[0] = 0x4d50504953544131ull;  // "MPPISTA1"
  h[1] = (uint64_t)c->L.TM;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(&h[2], c->base + c->L.off_iter, 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(&h[3], c->base + c->L.off_U64, (size_t)c->L.TM * 8, hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" int mppi_set_state(mppi_ctx *c, const void *buf, uint64_t len) {
  int rc = check_ctx(c);
  if (rc) return rc;
  const uint64_t need = 3 * 8 + (uint64_t)c->L.TM * 8;
  if (!buf || len < need) return fail(MPPI_EINVAL, "state buffer too small");
  const uint64_t *h = (const uint64_t *)buf;
  if (h[0] != 0x4d50504953544131ull || h[1] != (uint64_t)c->L.TM) return fail(MPPI_EINVAL, "state blob does not match this context");
  rc = mppi_set_controls(c, (const double *)&h[3], (uint64_t)c->L.TM);
  if (rc) return rc;
  HIP_TRY(hipMemcpy(c->base + c->L.off_iter, &h[2], 8, hipMemcpyHostToDevice));
  return MPPI_OK;
}

extern "C" int mppi_get_iteration(mppi_ctx *c, uint64_t *iteration) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!iteration) return fail(MPPI_EINVAL, "iteration is NULL");
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(iteration, c->base + c->L.off_iter, 8, hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" int mppi_debug_last(mppi_ctx *c, double *costs, double *rho, double *eta, double *dU) {
  int rc = check_ctx(c);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (costs) HIP_TRY(hipMemcpy(costs, c->base + c->L.off_S, (size_t)c->cfg.K * 8, hipMemcpyDeviceToHost));
  double head[2];
  HIP_TRY(hipMemcpy(head, c->base + c->L.off_dbg, 16, hipMemcpyDeviceToHost));
  if (rho) *rho = head[0];
  if (eta) *eta = head[1];
  if (dU) HIP_TRY(hipMemcpy(dU, c->base + c->L.off_dbg + 16, (size_t)c->L.TM * 8, hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" int mppi_debug_normals(mppi_ctx *c, uint64_t iteration, int32_t k0, int32_t nk, float *eps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!eps || k0 < 0 || nk < 1 || nk > (1 << 20)) return fail(MPPI_EINVAL, "bad k0/nk/eps");
  const int TM = c->L.TM, G = c->L.G;
  float *d = nullptr;
  HIP_TRY(hipMalloc((void **)&d, (size_t)nk * TM * 4));
  const int total = nk * G;
  hipLaunchKernelGGL(normals_kernel, dim3((total + 255) / 256), dim3(256), 0, c->stream, d, iteration,
                     (uint32_t)c->cfg.seed, (uint32_t)(c->cfg.seed >> 32), k0, nk, TM);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(eps, d, (size_t)nk * TM * 4, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "debug_normals");
  return MPPI_OK;
}

extern "C" int mppi_debug_philox(int32_t device, uint64_t seed, const uint32_t *counters, int32_t n, uint32_t *out) {
  if (!counters || !out || n < 1 || n > (1 << 24)) return fail(MPPI_EINVAL, "bad counters/out/n");
  int rc = set_device(device);
  if (rc) return rc;
  uint4 *dc = nullptr, *dout = nullptr;
  HIP_TRY(hipMalloc((void **)&dc, (size_t)n * 16));
  hipError_t e = hipMalloc((void **)&dout, (size_t)n * 16);
  if (e == hipSuccess) e = hipMemcpy(dc, counters, (size_t)n * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, dc, dout, n, (uint32_t)seed, (uint32_t)(seed >> 32));
    e = hipDeviceSynchronize();
  }
  if (e == hipSuccess) e = hipMemcpy(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost);
  (void)hipFree(dc);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return hip_fail(e, "debug_philox");
  return MPPI_OK;
}

extern "C" int mppi_debug_lane_groups(int32_t device, int32_t group, const float *a, const float *b, int32_t n_waves,
                                      float *out) {
  if (!a || !b || !out || n_waves < 1 || n_waves > 4096) return fail(MPPI_EINVAL, "bad a/b/out/n_waves");
  if (group != 4 && group != 16 && group != 32) return fail(MPPI_EINVAL, "group must be 4, 16 or 32");
  int rc = set_device(device);
  if (rc) return rc;
  const size_t n = (size_t)n_waves * kWave;
  float *d = nullptr;                                   // a | b | out (6 per lane)
  HIP_TRY(hipMalloc((void **)&d, n * 8 * sizeof(float)));
  hipError_t e = hipMemcpy(d, a, n * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d + n, b, n * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const void *fn = group == 4 ? (const void *)lane_groups_kernel<4>
                     : group == 16 ? (const void *)lane_groups_kernel<16> : (const void *)lane_groups_kernel<32>;
    const float *da = d, *db = d + n;
    float *dout = d + 2 * n;
    void *args[] = {(void *)&da, (void *)&db, (void *)&dout};
    e = hipLaunchKernel(fn, dim3(n_waves), dim3(kWave), args, 0, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e == hipSuccess) e = hipMemcpy(out, d + 2 * n, n * 6 * sizeof(float), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "debug_lane_groups");
  return MPPI_OK;
}

extern "C" int mppi_get_info(mppi_ctx *c, mppi_info *out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!out) return fail(MPPI_EINVAL, "out is NULL");
  const bool mlp = c->cfg.system == MPPI_SYS_QUADROTOR_MLP;
  out->rollout_lanes = mlp ? 4 : rollout_lps(&c->cfg);
  out->rollout_mode = mlp ? 0 : rollout_mode(c);
  out->rollout_blocks = c->L.n_roll_blocks;
  out->update_chunk = c->L.upd_chunk;
  out->update_blocks = c->L.fused ? 0 : c->L.n_kc * ((c->L.G + kUpdGroups - 1) / kUpdGroups);
  out->noise_groups = c->L.G;
  out->workspace_bytes = c->L.total;
  return MPPI_OK;
}

extern "C" int mppi_set_profiling(mppi_ctx *c, int32_t on) {
  int rc = check_ctx(c);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto &t : c->pending) { c->event_pool.push_back(t.a); c->event_pool.push_back(t.b); }
  c->pending.clear();
  c->profiling = on != 0;
  for (int k = 0; k < 3; ++k) { c->prof_ms[k] = 0.0; c->prof_n[k] = 0; }
  return MPPI_OK;
}

extern "C" int mppi_kernel_times(mppi_ctx *c, double *avg_ms, int64_t *count) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!avg_ms || !count) return fail(MPPI_EINVAL, "avg_ms and count must be non-NULL");
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto &t : c->pending) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    c->prof_ms[t.kind] += ms;
    c->prof_n[t.kind] += 1;
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->pending.clear();
  for (int k = 0; k < 3; ++k) {
    count[k] = c->prof_n[k];
    avg_ms[k] = c->prof_n[k] ? c->prof_ms[k] / (double)c->prof_n[k] : 0.0;
  }
  return MPPI_OK;
}

// ------------------------------------------------------ allocation-free control step
// Device memory of mppi_step_static: one file-scope array, which every GPU the library runs
// on holds at its own address until the process ends.  In host code the name `scratch` is a
// host-side stand-in, never a device address: its address on each device is looked up once
// (hipGetSymbolAddress, with that device current) and only that pointer is used.
static __device__ __align__(256) char scratch[MPPI_STATIC_SCRATCH_BYTES];

namespace mppi {
constexpr int kMaxStaticDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_dev[kMaxStaticDevices] = {};

// The device address of `scratch` on `dev` (the current device), looked up on the first call.
static int static_scratch(int dev, char **out) {
  if (dev < 0 || dev >= kMaxStaticDevices) return fail(MPPI_EINVAL, "device %d outside [0, %d)", dev, kMaxStaticDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(MPPI_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = (char *)p;
  }
  *out = g_scratch_dev[dev];
  return MPPI_OK;
}
}  // namespace mppi

extern "C" int mppi_step_static(const mppi_config *cfg, const double *x0, double *U, uint64_t *iteration,
                                int32_t n_iters, double *u0) {
  int rc = validate_config(cfg);
  if (rc) return rc;
  if (!x0 || !U || !iteration || !u0) return fail(MPPI_EINVAL, "x0, U, iteration and u0 must be non-NULL");
  if (n_iters < 1 || n_iters > 1000) return fail(MPPI_EINVAL, "n_iters=%d outside [1, 1000]", n_iters);
  if (cfg->system == MPPI_SYS_QUADROTOR_MLP)
    return fail(MPPI_EINVAL, "mppi_step_static: the learned dynamics need device buffers of their own");
  if (!finite_all(x0, cfg->n_state) || !finite_all(U, cfg->T * cfg->n_ctrl))
    return fail(MPPI_EINVAL, "x0 or U has non-finite entries");
  rc = set_device(cfg->device);
  if (rc) return rc;
  char *base = nullptr;
  rc = static_scratch(cfg->device, &base);
  if (rc) return rc;
  // a context on the stack: its containers stay empty (no graphs, no profiling events)
  mppi_ctx c;
  init_host_state(&c, cfg);
  if (c.L.total > MPPI_STATIC_SCRATCH_BYTES)
    return fail(MPPI_EINVAL, "mppi_step_static: K=%d, T=%d needs %llu B of device state, the static scratch holds %llu B",
                cfg->K, cfg->T, (unsigned long long)c.L.total, (unsigned long long)MPPI_STATIC_SCRATCH_BYTES);
  c.base = base;
  c.stream = (hipStream_t)cfg->stream;
  c.cfg.use_graph = 0;
  c.cfg.workspace = nullptr;
  // the previous call on this device is complete (calls block), so the system data, the
  // sequence and the counters can be rewritten; what the kernels expect at zero is cleared
  rc = build_params(&c);
  if (!rc) rc = prepare_system(&c);
  if (rc) return rc;
  const int T = cfg->T, m = cfg->n_ctrl, n = cfg->n_state;
  float U32[kMaxTM];
  for (int i = 0; i < T * m; ++i) U32[i] = (float)U[i];
  HIP_TRY(hipMemsetAsync(base, 0, c.L.off_U64, c.stream));
  HIP_TRY(hipMemcpyAsync(base + c.L.off_x0, x0, (size_t)n * 8, hipMemcpyHostToDevice, c.stream));
  HIP_TRY(hipMemcpyAsync(base + c.L.off_iter, iteration, 8, hipMemcpyHostToDevice, c.stream));
  HIP_TRY(hipMemcpyAsync(base + c.L.off_U64, U, (size_t)T * m * 8, hipMemcpyHostToDevice, c.stream));
  HIP_TRY(hipMemcpyAsync(base + c.L.off_U32, U32, (size_t)T * m * 4, hipMemcpyHostToDevice, c.stream));
  double *d_res = (double *)(base + c.L.off_res);
  rc = enqueue_iterations(&c, (const double *)(base + c.L.off_x0), n_iters, d_res, c.stream, nullptr);
  if (rc) return rc;
  double res[8];
  HIP_TRY(hipMemcpyAsync(res, d_res, sizeof(res), hipMemcpyDeviceToHost, c.stream));
  HIP_TRY(hipMemcpyAsync(U, base + c.L.off_U64, (size_t)T * m * 8, hipMemcpyDeviceToHost, c.stream));
  HIP_TRY(hipMemcpyAsync(iteration, base + c.L.off_iter, 8, hipMemcpyDeviceToHost, c.stream));
  HIP_TRY(hipStreamSynchronize(c.stream));
  std::memcpy(u0, res, (size_t)m * sizeof(double));
  int count;
  std::memcpy(&count, res + 4, sizeof(int));
  if (count != 0) return fail(MPPI_ENUMERIC, "an iteration had no sample with a finite path cost; U was left unchanged");
  return MPPI_OK;
}
