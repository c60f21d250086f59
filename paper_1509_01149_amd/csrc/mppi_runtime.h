// Host-side context of libmppi (internal; the public contract is include/mppi.h).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mppi.h"
#include "mppi_batched.h"

namespace mppi {

// Offsets (bytes) of every device buffer inside one workspace allocation.
struct Layout {
  int TM, G, n_roll_blocks, n_kc, upd_chunk;
  bool fused;                                        // two kernels per iteration (kFused)
  bool multi;                                        // multi-block finalize (always when fused)
  int n_fin_blocks;                                  // finalize blocks: 1, or ceil(TM / kFinOut) multi
  uint64_t off_shadow;                               // multi only: the master as the finalize reads it
  uint64_t off_basis;                                // multi only: the plant basis [M + 1][N] of a plant step
  bool ctg_fold;                                     // cost-to-go, step-split: rollout blocks' step minima
  uint64_t off_blk_tail;                             //   [n_roll_blocks][T] (no per-step minimum pass)
  uint64_t off_x0, off_res, off_iter, off_U64, off_U32, off_S, off_blk_min, off_eta_part, off_part, off_dbg,
      off_pre, off_rho_step, off_sys, off_extra, extra_bytes, total;   // off_pre/off_rho_step: cost-to-go only
  uint64_t off_rho;                                  // the iteration's minimum path cost
};

struct MlpState;  // learned-dynamics extension (mppi_mlp.hip)

}  // namespace mppi

struct mppi_ctx {
  mppi_config cfg;                 // copy; its host pointers are cleared after create
  mppi::Layout L;
  char *base = nullptr;            // device workspace
  bool owns_ws = false;
  hipStream_t stream = nullptr;
  bool owns_stream = false;
  hipStream_t cap_stream = nullptr;
  char *pinned = nullptr;          // 4 KiB pinned staging for x0 / results
  double L64[16] = {0};            // chol(sigma)
  double Ls[16] = {0};             // A chol(sigma), A = diag(sqrt(nu_j))
  double Mq[16] = {0};             // (R - A^-1 R A^-1) / 2
  double R[16] = {0};
  double u_init[4] = {0};
  int seen_numeric = 0;
  mppi::LinearParams linear;
  mppi::CartPoleSys::Params cartpole;
  mppi::SwingUpSys::Params swingup;
  mppi::BicycleSys::Params bicycle;
  mppi::QuadrotorSys::Params quad;
  mppi::MlpState *mlp = nullptr;
  // captured graphs keyed by (n_steps, n_iters, x0, u0, plant state)
  std::map<std::tuple<int, int, const void *, const void *, const void *>, hipGraphExec_t> graphs;
  // profiling: pending (kind, start, stop) event triples and accumulated totals
  bool profiling = false;
  struct Timed { int kind; hipEvent_t a, b; };
  std::vector<Timed> pending;
  std::vector<hipEvent_t> event_pool;
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_n[3] = {0, 0, 0};
  template <int M>
  const mppi::LinearParams &linear_as() const { return linear; }
};

namespace mppi {
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate_config(const mppi_config *c);
void compute_layout(const mppi_config *c, Layout *L);
bool rollout_split(const mppi_config *c);
bool fused_available(const mppi_config *c);
int rollout_lps(const mppi_config *c);
int enqueue_iterations(mppi_ctx *c, const double *x0_dev, int n_iters, double *u0_dev, hipStream_t s,
                       double *plant_x);
int run_iterations(mppi_ctx *c, const double *x0_dev, int n_iters, double *u0_dev, double *plant_x,
                   int n_steps = 1);
size_t ctx_rollout_lds(const mppi_ctx *c);
void fill_desc(mppi_ctx *c, CtrlDesc *d);
int set_device(int dev);

// learned-dynamics hooks (mppi_mlp.hip)
uint64_t extra_workspace_bytes(const mppi_config *c);
int init_extra(mppi_ctx *c, const mppi_config *cfg);
void destroy_extra(mppi_ctx *c);
int launch_mlp_rollout(mppi_ctx *c, const IterArgs &a, hipStream_t s);
int timed_launch(mppi_ctx *c, int kind, const void *fn, dim3 grid, dim3 block, void **args, size_t lds,
                 hipStream_t s);
int prepare_mlp_rollout(mppi_ctx *c);
size_t mlp_rollout_lds(const mppi_ctx *c);
}  // namespace mppi
