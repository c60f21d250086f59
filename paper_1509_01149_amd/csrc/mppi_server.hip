// Serving runtime: continuous batching of many MPPI controllers on one GPU
// (contract in include/mppi.h, "Serving").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mppi.h"
#include "mppi_runtime.h"

using namespace mppi;

namespace {

// rollout instantiations: linear m=1,2,4, cart-pole, bicycle, quadrotor, swing-up, quadrotor
// with the crash indicator; kinds 8 + (0, 1, 2, 3, 4, 6) are the step-split systems at 16
// lanes per sample (at 4 below that), kind 16 + 4 the bicycle at 32; kFusedKind + k is the
// fused variant of kind k (the step-split kinds and the quadrotor's)
constexpr int kWide = 8;
constexpr int kFusedKind = 24;
constexpr int kKinds = 48;
using KindMask = uint64_t;
static_assert(kKinds <= 64, "kind sets are 64-bit masks");

int kind_of(const mppi_config &c) {
  if (c.system == MPPI_SYS_QUADROTOR && ((const mppi_quadrotor_params *)c.params)->crash_cost > 0) return 7;
  const int lps = rollout_split(&c) ? rollout_lps(&c) : 0;
  const int wide = lps == 32 ? 2 * kWide : (lps == 16 ? kWide : 0);
  switch (c.system) {
    case MPPI_SYS_LINEAR: return wide + (c.n_ctrl == 1 ? 0 : (c.n_ctrl == 2 ? 1 : 2));
    case MPPI_SYS_CARTPOLE: return wide + 3;
    case MPPI_SYS_BICYCLE: return wide + 4;
    case MPPI_SYS_CARTPOLE_SWINGUP: return wide + 6;
    default: return 5;
  }
}

struct Request {
  uint64_t id;
  double t_arrival;
  double x0[16];
};

struct Slot {
  bool used = false;
  mppi_ctx *ctx = nullptr;
  std::deque<Request> q;
  bool busy = false;
  uint64_t bytes = 0;
  int kind = 0;
  int m = 0;
  int n_roll = 0, n_upd = 0, n_fin = 1;
  size_t lds = 0;
  int64_t rollout_steps = 0;
};

struct Entry {
  int slot;
  uint64_t id;
  double t_arrival;
};

// Per-stream batch buffers: plan + staged start states (uploaded), results (downloaded).
// A batch that mixes system types runs each type's rollout on its own stream (the batch
// stream and kSide side streams forked from it), so the types' kernels fill the device
// together instead of one after the other; the update and finalize join on the batch
// stream.
constexpr int kSide = 2;
struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t roll[kKinds] = {};
  hipGraphNode_t upd = nullptr, fin = nullptr, down = nullptr;
};
constexpr size_t kMaxBatchGraphs = 64;   // kind sets kept per stream

struct Batch {
  hipStream_t stream = nullptr;
  hipStream_t side[kSide] = {nullptr, nullptr};
  hipEvent_t fork = nullptr, join[kSide] = {nullptr, nullptr};
  hipEvent_t done = nullptr;
  bool active = false;
  char *h = nullptr, *d = nullptr;
  size_t off_items = 0, off_sel = 0, off_proll = 0, off_pupd = 0, off_pfin = 0, off_x0 = 0, off_out = 0, bytes = 0;
  std::vector<Entry> entries;
  // BATCHED_GRAPH: one instantiated graph per set of rollout kinds a batch holds (the plan upload,
  // the kinds' rollouts as parallel branches, the update, the finalize and the result
  // download); a launch rewrites the kernel nodes' grids and counts for its batch
  std::map<KindMask, BatchGraph> graphs;
};


struct Result {
  uint64_t id;
  double u0[4];
  int status;
  double t_done;
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct mppi_server {
  mppi_server_config cfg;
  std::mutex mu;
  std::chrono::steady_clock::time_point t0;
  std::vector<Slot> slots;
  uint64_t used = 0;
  CtrlDesc *d_descs = nullptr;
  std::vector<Batch> batches;
  std::deque<int> fifo;            // PLAIN: slots in submission order
  std::vector<Result> done;
  int rr = 0;                      // round-robin start for batch formation
  size_t lds_set[kKinds] = {0};
  int64_t n_done = 0, n_batches = 0, n_batched_req = 0, steps_done = 0;
  int queued = 0, inflight = 0;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

// The rollout instantiation of each kind (see kind_of).
const void *roll_fn(int k) {
  switch (k) {
    case kFusedKind + 0: return (const void *)rollout_batched<LinearSys<1>, 4, kStepSplit | kFused>;
    case kFusedKind + 1: return (const void *)rollout_batched<LinearSys<2>, 4, kStepSplit | kFused>;
    case kFusedKind + 2: return (const void *)rollout_batched<LinearSys<4>, 4, kStepSplit | kFused>;
    case kFusedKind + 3: return (const void *)rollout_batched<CartPoleSys, 4, kStepSplit | kFused>;
    case kFusedKind + 4: return (const void *)rollout_batched<BicycleSys, 4, kStepSplit | kFused>;
    case kFusedKind + 5: return (const void *)rollout_batched<QuadrotorSys, QuadrotorSys::kLPS, kFused>;
    case kFusedKind + 6: return (const void *)rollout_batched<SwingUpSys, 4, kStepSplit | kFused>;
    case kFusedKind + 7: return (const void *)rollout_batched<QuadrotorSys, QuadrotorSys::kLPS, kCrashOn | kFused>;
    case kFusedKind + kWide + 0: return (const void *)rollout_batched<LinearSys<1>, 16, kStepSplit | kFused>;
    case kFusedKind + kWide + 1: return (const void *)rollout_batched<LinearSys<2>, 16, kStepSplit | kFused>;
    case kFusedKind + kWide + 2: return (const void *)rollout_batched<LinearSys<4>, 16, kStepSplit | kFused>;
    case kFusedKind + kWide + 3: return (const void *)rollout_batched<CartPoleSys, 16, kStepSplit | kFused>;
    case kFusedKind + kWide + 4: return (const void *)rollout_batched<BicycleSys, 16, kStepSplit | kFused>;
    case kFusedKind + kWide + 6: return (const void *)rollout_batched<SwingUpSys, 16, kStepSplit | kFused>;
    case kFusedKind + 2 * kWide + 4: return (const void *)rollout_batched<BicycleSys, 32, kStepSplit | kFused>;
    case 0: return (const void *)rollout_batched<LinearSys<1>, 4, kStepSplit>;
    case 1: return (const void *)rollout_batched<LinearSys<2>, 4, kStepSplit>;
    case 2: return (const void *)rollout_batched<LinearSys<4>, 4, kStepSplit>;
    case 3: return (const void *)rollout_batched<CartPoleSys, 4, kStepSplit>;
    case 4: return (const void *)rollout_batched<BicycleSys, 4, kStepSplit>;
    case 5: return (const void *)rollout_batched<QuadrotorSys, QuadrotorSys::kLPS, 0>;
    case 6: return (const void *)rollout_batched<SwingUpSys, 4, kStepSplit>;
    case 7: return (const void *)rollout_batched<QuadrotorSys, QuadrotorSys::kLPS, kCrashOn>;
    case kWide + 0: return (const void *)rollout_batched<LinearSys<1>, 16, kStepSplit>;
    case kWide + 1: return (const void *)rollout_batched<LinearSys<2>, 16, kStepSplit>;
    case kWide + 2: return (const void *)rollout_batched<LinearSys<4>, 16, kStepSplit>;
    case kWide + 3: return (const void *)rollout_batched<CartPoleSys, 16, kStepSplit>;
    case kWide + 4: return (const void *)rollout_batched<BicycleSys, 16, kStepSplit>;
    case kWide + 6: return (const void *)rollout_batched<SwingUpSys, 16, kStepSplit>;
    case 2 * kWide + 4: return (const void *)rollout_batched<BicycleSys, 32, kStepSplit>;
    default: return nullptr;
  }
}

// Dynamic LDS above the default needs the kernel's attribute raised first (once per size).
int ensure_lds(mppi_server *s, int k, size_t lds) {
  if (lds > s->lds_set[k]) {
    const hipError_t e = hipFuncSetAttribute(roll_fn(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "rollout LDS attribute");
    s->lds_set[k] = lds;
  }
  return MPPI_OK;
}

// The kernel arguments of one batch, in the launch order of the kernels.
struct BatchArgs {
  const CtrlDesc *descs;
  const WorkItem *items;
  const int *sel[kKinds];
  const int *proll[kKinds];
  const int *pupd;
  const int *pfin;
  int count[kKinds];
  int nb;
};

hipKernelNodeParams roll_params(BatchArgs &a, int k, int total, size_t lds, void **argv) {
  argv[0] = (void *)&a.descs;
  argv[1] = (void *)&a.items;
  argv[2] = (void *)&a.sel[k];
  argv[3] = (void *)&a.proll[k];
  argv[4] = (void *)&a.count[k];
  hipKernelNodeParams p{};
  p.func = (void *)roll_fn(k);
  p.gridDim = dim3(total > 0 ? total : 1);
  p.blockDim = dim3(kBlock);
  p.sharedMemBytes = (unsigned)lds;
  p.kernelParams = argv;
  p.extra = nullptr;
  return p;
}

hipKernelNodeParams upd_params(BatchArgs &a, int blocks, void **argv) {
  argv[0] = (void *)&a.descs;
  argv[1] = (void *)&a.items;
  argv[2] = (void *)&a.pupd;
  argv[3] = (void *)&a.nb;
  hipKernelNodeParams p{};
  p.func = (void *)update_batched;
  p.gridDim = dim3(blocks > 0 ? blocks : 1);
  p.blockDim = dim3(kBlock);
  p.kernelParams = argv;
  return p;
}

hipKernelNodeParams fin_params(BatchArgs &a, int blocks, void **argv) {
  argv[0] = (void *)&a.descs;
  argv[1] = (void *)&a.items;
  argv[2] = (void *)&a.pfin;
  argv[3] = (void *)&a.nb;
  hipKernelNodeParams p{};
  p.func = (void *)finalize_batched;
  p.gridDim = dim3(blocks > 0 ? blocks : 1);
  p.blockDim = dim3(kFinBlock);
  p.kernelParams = argv;
  return p;
}

void destroy_graph(BatchGraph &G) {
  if (G.exec) (void)hipGraphExecDestroy(G.exec);
  if (G.graph) (void)hipGraphDestroy(G.graph);
  G = BatchGraph();
}

// The graph of a batch stream for one set of rollout kinds: upload -> rollouts (one branch
// per kind) -> update -> finalize -> download.  Grids and counts are placeholders until a
// launch sets them.
int build_graph(mppi_server *s, Batch &b, KindMask mask, BatchArgs &a, BatchGraph &G) {
  const int B = s->cfg.max_batch;
  hipError_t e = hipGraphCreate(&G.graph, 0);
  hipGraphNode_t up = nullptr;
  if (e == hipSuccess) e = hipGraphAddMemcpyNode1D(&up, G.graph, nullptr, 0, b.d, b.h, b.off_out, hipMemcpyHostToDevice);
  std::vector<hipGraphNode_t> rolls;
  for (int k = 0; k < kKinds && e == hipSuccess; ++k) {
    if (!(mask >> k & 1ull)) continue;
    void *argv[5];
    const hipKernelNodeParams p = roll_params(a, k, 1, 0, argv);
    e = hipGraphAddKernelNode(&G.roll[k], G.graph, &up, 1, &p);
    rolls.push_back(G.roll[k]);
  }
  void *uargv[4], *fargv[4];
  if (e == hipSuccess) {
    const hipKernelNodeParams p = upd_params(a, 1, uargv);
    e = hipGraphAddKernelNode(&G.upd, G.graph, rolls.data(), rolls.size(), &p);
  }
  if (e == hipSuccess) {
    const hipKernelNodeParams p = fin_params(a, 1, fargv);
    e = hipGraphAddKernelNode(&G.fin, G.graph, &G.upd, 1, &p);
  }
  if (e == hipSuccess)
    e = hipGraphAddMemcpyNode1D(&G.down, G.graph, &G.fin, 1, b.h + b.off_out, b.d + b.off_out,
                                (size_t)B * 8 * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    destroy_graph(G);
    return hip_fail(e, "batch graph");
  }
  return MPPI_OK;
}

int launch_batched(mppi_server *s, Batch &b, const std::vector<int> &sl) {
  const int B = s->cfg.max_batch;
  const int nb = (int)sl.size();
  auto *items = (WorkItem *)(b.h + b.off_items);
  auto *sel = (int *)(b.h + b.off_sel);
  auto *proll = (int *)(b.h + b.off_proll);
  auto *pupd = (int *)(b.h + b.off_pupd);
  auto *pfin = (int *)(b.h + b.off_pfin);
  auto *x0 = (double *)(b.h + b.off_x0);
  int cnt[kKinds] = {0};
  size_t lds[kKinds] = {0};
  for (int k = 0; k < kKinds; ++k) proll[k * (B + 1)] = 0;
  pupd[0] = 0;
  pfin[0] = 0;
  b.entries.clear();
  for (int j = 0; j < nb; ++j) {
    Slot &S = s->slots[sl[j]];
    Request r = S.q.front();
    S.q.pop_front();
    S.busy = true;
    std::memcpy(x0 + 16 * j, r.x0, sizeof(r.x0));
    items[j].desc = sl[j];
    items[j].pad = 0;
    items[j].x0 = (const double *)(b.d + b.off_x0) + 16 * j;
    items[j].out = (double *)(b.d + b.off_out) + 8 * j;
    const int k = S.kind;
    sel[k * B + cnt[k]] = j;
    proll[k * (B + 1) + cnt[k] + 1] = proll[k * (B + 1) + cnt[k]] + S.n_roll;
    cnt[k] += 1;
    lds[k] = std::max(lds[k], S.lds);
    pupd[j + 1] = pupd[j] + S.n_upd;
    pfin[j + 1] = pfin[j] + S.n_fin;
    b.entries.push_back({sl[j], r.id, r.t_arrival});
  }
  BatchArgs a;
  a.descs = s->d_descs;
  a.items = (const WorkItem *)(b.d + b.off_items);
  a.pupd = (const int *)(b.d + b.off_pupd);
  a.pfin = (const int *)(b.d + b.off_pfin);
  a.nb = nb;
  KindMask mask = 0;
  int kinds[kKinds], nk = 0;
  for (int k = 0; k < kKinds; ++k) {
    a.sel[k] = (const int *)(b.d + b.off_sel) + k * B;
    a.proll[k] = (const int *)(b.d + b.off_proll) + k * (B + 1);
    a.count[k] = cnt[k];
    if (cnt[k]) {
      kinds[nk++] = k;
      mask |= 1ull << k;
      const int rc = ensure_lds(s, k, lds[k]);
      if (rc) return rc;
    }
  }
  hipError_t e = hipSuccess;
  if (s->cfg.mode == MPPI_SERVE_BATCHED_GRAPH) {
    auto it = b.graphs.find(mask);
    if (it == b.graphs.end()) {
      if (b.graphs.size() >= kMaxBatchGraphs) {      // bounded cache (this stream is idle)
        for (auto &kv : b.graphs) destroy_graph(kv.second);
        b.graphs.clear();
      }
      BatchGraph G;
      const int rc = build_graph(s, b, mask, a, G);
      if (rc) return rc;
      it = b.graphs.emplace(mask, G).first;
    }
    BatchGraph &G = it->second;
    for (int i = 0; i < nk && e == hipSuccess; ++i) {
      const int k = kinds[i];
      void *argv[5];
      const hipKernelNodeParams p = roll_params(a, k, proll[k * (B + 1) + cnt[k]], lds[k], argv);
      e = hipGraphExecKernelNodeSetParams(G.exec, G.roll[k], &p);
    }
    void *uargv[4], *fargv[4];
    if (e == hipSuccess) {
      const hipKernelNodeParams p = upd_params(a, pupd[nb], uargv);
      e = hipGraphExecKernelNodeSetParams(G.exec, G.upd, &p);
    }
    if (e == hipSuccess) {
      const hipKernelNodeParams p = fin_params(a, pfin[nb], fargv);
      e = hipGraphExecKernelNodeSetParams(G.exec, G.fin, &p);
    }
    if (e == hipSuccess)
      e = hipGraphExecMemcpyNodeSetParams1D(G.exec, G.down, b.h + b.off_out, b.d + b.off_out,
                                            (size_t)nb * 8 * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipGraphLaunch(G.exec, b.stream);
    if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
    if (e != hipSuccess) return hip_fail(e, "batch graph launch");
  } else {
    // direct launches: one stream per system type present (the batch stream first, then
    // the side streams), joined before the update
    e = hipMemcpyAsync(b.d, b.h, b.off_out, hipMemcpyHostToDevice, b.stream);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    const int n_side = std::min(nk - 1, kSide);
    if (n_side > 0) {
      e = hipEventRecord(b.fork, b.stream);
      for (int i = 0; i < n_side && e == hipSuccess; ++i) e = hipStreamWaitEvent(b.side[i], b.fork, 0);
      if (e != hipSuccess) return hip_fail(e, "batch fork");
    }
    for (int i = 0; i < nk && e == hipSuccess; ++i) {
      const int k = kinds[i];
      const hipStream_t st = i == 0 ? b.stream : b.side[(i - 1) % kSide];
      void *argv[5];
      const hipKernelNodeParams p = roll_params(a, k, proll[k * (B + 1) + cnt[k]], lds[k], argv);
      e = hipLaunchKernel(p.func, p.gridDim, p.blockDim, p.kernelParams, p.sharedMemBytes, st);
    }
    if (e != hipSuccess) return hip_fail(e, "batch rollout launch");
    for (int i = 0; i < n_side; ++i) {
      e = hipEventRecord(b.join[i], b.side[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b.stream, b.join[i], 0);
      if (e != hipSuccess) return hip_fail(e, "batch join");
    }
    void *uargv[4], *fargv[4];
    if (pupd[nb] > 0) {                             // fused controllers have no update blocks
      const hipKernelNodeParams pu = upd_params(a, pupd[nb], uargv);
      e = hipLaunchKernel(pu.func, pu.gridDim, pu.blockDim, pu.kernelParams, 0, b.stream);
    }
    const hipKernelNodeParams pf = fin_params(a, pfin[nb], fargv);
    if (e == hipSuccess) e = hipLaunchKernel(pf.func, pf.gridDim, pf.blockDim, pf.kernelParams, 0, b.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.h + b.off_out, b.d + b.off_out, (size_t)nb * 8 * sizeof(double),
                                            hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
  }
  b.active = true;
  s->n_batches += 1;
  s->n_batched_req += nb;
  s->queued -= nb;
  s->inflight += nb;
  return MPPI_OK;
}

// PLAIN: one controller step through its own captured single-controller graph.
int launch_plain(mppi_server *s, Batch &b, int slot) {
  Slot &S = s->slots[slot];
  Request r = S.q.front();
  S.q.pop_front();
  S.busy = true;
  mppi_ctx *c = S.ctx;
  double *hx = (double *)(b.h + b.off_x0);
  std::memcpy(hx, r.x0, sizeof(r.x0));
  double *d_x0 = (double *)(c->base + c->L.off_x0);
  double *d_res = (double *)(c->base + c->L.off_res);
  hipError_t e = hipMemcpyAsync(d_x0, hx, 16 * sizeof(double), hipMemcpyHostToDevice, b.stream);
  if (e != hipSuccess) return hip_fail(e, "plain upload");
  int rc = run_iterations(c, d_x0, 1, d_res, nullptr);
  if (rc) return rc;
  e = hipMemcpyAsync(b.h + b.off_out, d_res, 8 * sizeof(double), hipMemcpyDeviceToHost, b.stream);
  if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
  if (e != hipSuccess) return hip_fail(e, "plain launch");
  b.entries.clear();
  b.entries.push_back({slot, r.id, r.t_arrival});
  b.active = true;
  s->n_batches += 1;
  s->n_batched_req += 1;
  s->queued -= 1;
  s->inflight += 1;
  return MPPI_OK;
}

int harvest(mppi_server *s, Batch &b) {
  hipError_t e = hipEventQuery(b.done);
  if (e == hipErrorNotReady) return MPPI_OK;
  if (e != hipSuccess) return hip_fail(e, "batch completion");
  const double t = s->now();
  const double *out = (const double *)(b.h + b.off_out);
  for (size_t j = 0; j < b.entries.size(); ++j) {
    const Entry &en = b.entries[j];
    Slot &S = s->slots[en.slot];
    Result r;
    r.id = en.id;
    r.t_done = t;
    for (int i = 0; i < 4; ++i) r.u0[i] = i < S.m ? out[8 * j + i] : 0.0;
    if (s->cfg.mode == MPPI_SERVE_PLAIN) {
      int cnt;
      std::memcpy(&cnt, out + 4, sizeof(int));
      r.status = cnt != S.ctx->seen_numeric ? MPPI_ENUMERIC : MPPI_OK;
      S.ctx->seen_numeric = cnt;
    } else {
      r.status = out[8 * j + 4] != 0.0 ? MPPI_ENUMERIC : MPPI_OK;
    }
    s->done.push_back(r);
    S.busy = false;
    s->n_done += 1;
    s->steps_done += S.rollout_steps;
    s->inflight -= 1;
  }
  b.entries.clear();
  b.active = false;
  return MPPI_OK;
}

int progress(mppi_server *s) {
  for (auto &b : s->batches)
    if (b.active) {
      int rc = harvest(s, b);
      if (rc) return rc;
    }
  for (auto &b : s->batches) {
    if (b.active) continue;
    if (s->cfg.mode == MPPI_SERVE_PLAIN) {
      while (!s->fifo.empty() && (!s->slots[s->fifo.front()].used || s->slots[s->fifo.front()].q.empty()))
        s->fifo.pop_front();
      if (s->fifo.empty()) break;
      const int slot = s->fifo.front();
      if (s->slots[slot].busy) break;   // keep arrival order
      s->fifo.pop_front();
      int rc = launch_plain(s, b, slot);
      if (rc) return rc;
      continue;
    }
    std::vector<int> sl;
    const int n = (int)s->slots.size();
    for (int i = 0; i < n && (int)sl.size() < s->cfg.max_batch; ++i) {
      const int k = (s->rr + i) % n;
      const Slot &S = s->slots[k];
      if (S.used && !S.busy && !S.q.empty()) sl.push_back(k);
    }
    if (sl.empty()) break;
    s->rr = (sl.back() + 1) % n;
    int rc = launch_batched(s, b, sl);
    if (rc) return rc;
  }
  return MPPI_OK;
}

int check_srv(mppi_server *s) {
  if (!s) return fail(MPPI_EINVAL, "server is NULL");
  hipError_t e = hipSetDevice(s->cfg.device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return MPPI_OK;
}

}  // namespace

extern "C" int mppi_server_create(const mppi_server_config *cfg, mppi_server **out) {
  if (!cfg || !out) return fail(MPPI_EINVAL, "cfg and out must be non-NULL");
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 4096) return fail(MPPI_EINVAL, "max_slots outside [1, 4096]");
  if (cfg->max_inflight < 1 || cfg->max_inflight > 8) return fail(MPPI_EINVAL, "max_inflight outside [1, 8]");
  if (cfg->max_batch < 1 || cfg->max_batch > cfg->max_slots) return fail(MPPI_EINVAL, "max_batch outside [1, max_slots]");
  if (cfg->mode != MPPI_SERVE_BATCHED && cfg->mode != MPPI_SERVE_PLAIN && cfg->mode != MPPI_SERVE_BATCHED_GRAPH)
    return fail(MPPI_EINVAL, "unknown mode");
  int rc = set_device(cfg->device);
  if (rc) return rc;
  auto *s = new mppi_server();
  s->cfg = *cfg;
  if (cfg->mode == MPPI_SERVE_PLAIN) { s->cfg.max_inflight = 1; s->cfg.max_batch = 1; }
  s->t0 = std::chrono::steady_clock::now();
  s->slots.resize(cfg->max_slots);
  hipError_t e = hipMalloc((void **)&s->d_descs, sizeof(CtrlDesc) * cfg->max_slots);
  if (e != hipSuccess) { delete s; return fail(MPPI_ENOMEM, "descriptor table: %s", hipGetErrorString(e)); }
  const int B = s->cfg.max_batch;
  s->batches.resize(s->cfg.max_inflight);
  for (auto &b : s->batches) {
    b.off_items = 0;
    b.off_sel = al(b.off_items + sizeof(WorkItem) * B);
    b.off_proll = al(b.off_sel + sizeof(int) * kKinds * B);
    b.off_pupd = al(b.off_proll + sizeof(int) * kKinds * (B + 1));
    b.off_pfin = al(b.off_pupd + sizeof(int) * (B + 1));
    b.off_x0 = al(b.off_pfin + sizeof(int) * (B + 1));
    b.off_out = al(b.off_x0 + sizeof(double) * 16 * B);
    b.bytes = al(b.off_out + sizeof(double) * 8 * B);
    e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
    for (int i = 0; i < kSide && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&b.side[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b.h, b.bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void **)&b.d, b.bytes);
    if (e != hipSuccess) { mppi_server_destroy(s); return hip_fail(e, "server stream buffers"); }
    std::memset(b.h, 0, b.bytes);
  }
  *out = s;
  return MPPI_OK;
}

extern "C" int mppi_server_destroy(mppi_server *s) {
  if (!s) return MPPI_OK;
  (void)hipSetDevice(s->cfg.device);
  for (auto &b : s->batches) {
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    for (auto st : b.side) if (st) (void)hipStreamSynchronize(st);
  }
  for (auto &S : s->slots) if (S.ctx) mppi_destroy(S.ctx);
  for (auto &b : s->batches) {
    for (auto &kv : b.graphs) destroy_graph(kv.second);
    if (b.h) (void)hipHostFree(b.h);
    if (b.d) (void)hipFree(b.d);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.fork) (void)hipEventDestroy(b.fork);
    for (int i = 0; i < kSide; ++i) {
      if (b.join[i]) (void)hipEventDestroy(b.join[i]);
      if (b.side[i]) (void)hipStreamDestroy(b.side[i]);
    }
    if (b.stream) (void)hipStreamDestroy(b.stream);
  }
  if (s->d_descs) (void)hipFree(s->d_descs);
  delete s;
  return MPPI_OK;
}

extern "C" int mppi_server_admit(mppi_server *s, const mppi_config *cfg, int32_t *slot) {
  int rc = check_srv(s);
  if (rc) return rc;
  if (!cfg || !slot) return fail(MPPI_EINVAL, "cfg and slot must be non-NULL");
  if (cfg->system == MPPI_SYS_QUADROTOR_MLP) return fail(MPPI_EINVAL, "the server runs the analytic systems");
  if (cfg->weighting != MPPI_WEIGHT_PATH) return fail(MPPI_EINVAL, "the server runs path-cost weighting only");
  mppi_config c = *cfg;
  std::lock_guard<std::mutex> lk(s->mu);
  uint64_t bytes = 0;
  rc = mppi_workspace_bytes(&c, &bytes);
  if (rc) return rc;
  int free_slot = -1;
  for (int i = 0; i < (int)s->slots.size(); ++i)
    if (!s->slots[i].used) { free_slot = i; break; }
  if (free_slot < 0) return fail(MPPI_EBUSY, "no free slot");
  if (s->used + bytes > s->cfg.hbm_budget_bytes)
    return fail(MPPI_EBUSY, "HBM budget: %llu + %llu > %llu bytes", (unsigned long long)s->used,
                (unsigned long long)bytes, (unsigned long long)s->cfg.hbm_budget_bytes);
  c.device = s->cfg.device;
  c.stream = s->batches[0].stream;
  c.workspace = nullptr;
  c.workspace_bytes = 0;
  c.use_graph = 1;
  mppi_ctx *ctx = nullptr;
  rc = mppi_create(&c, &ctx);
  if (rc) return rc;
  CtrlDesc d;
  fill_desc(ctx, &d);
  hipError_t e = hipMemcpy(s->d_descs + free_slot, &d, sizeof(d), hipMemcpyHostToDevice);
  if (e != hipSuccess) { mppi_destroy(ctx); return hip_fail(e, "descriptor upload"); }
  Slot &S = s->slots[free_slot];
  S = Slot();
  S.used = true;
  S.ctx = ctx;
  S.bytes = bytes;
  S.kind = kind_of(c) + (ctx->L.fused ? kFusedKind : 0);
  S.m = c.n_ctrl;
  S.n_roll = ctx->L.n_roll_blocks + (ctx->L.multi ? 1 : 0);   // the shadow block
  S.n_upd = ctx->L.fused ? 0 : ctx->L.n_kc * ((ctx->L.G + kUpdGroups - 1) / kUpdGroups);
  S.n_fin = ctx->L.multi ? (ctx->L.n_fin_blocks + 3) / 4 : 1;   // four multi-block finalize blocks per block
  S.lds = ctx_rollout_lds(ctx);
  S.rollout_steps = (int64_t)c.K * c.T;
  s->used += bytes;
  *slot = free_slot;
  return MPPI_OK;
}

extern "C" int mppi_server_release(mppi_server *s, int32_t slot) {
  int rc = check_srv(s);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  if (slot < 0 || slot >= (int)s->slots.size() || !s->slots[slot].used) return fail(MPPI_ENOTFOUND, "unknown slot %d", slot);
  Slot &S = s->slots[slot];
  if (S.busy || !S.q.empty()) return fail(MPPI_EBUSY, "slot %d has queued or in-flight steps", slot);
  mppi_destroy(S.ctx);
  s->used -= S.bytes;
  S = Slot();
  return MPPI_OK;
}

extern "C" int mppi_server_submit(mppi_server *s, int32_t slot, const double *x0, uint64_t req_id, double t_arrival) {
  int rc = check_srv(s);
  if (rc) return rc;
  if (!x0) return fail(MPPI_EINVAL, "x0 is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (slot < 0 || slot >= (int)s->slots.size() || !s->slots[slot].used) return fail(MPPI_ENOTFOUND, "unknown slot %d", slot);
  Slot &S = s->slots[slot];
  Request r;
  r.id = req_id;
  r.t_arrival = t_arrival;
  std::memset(r.x0, 0, sizeof(r.x0));
  for (int i = 0; i < S.ctx->cfg.n_state; ++i) {
    if (!std::isfinite(x0[i])) return fail(MPPI_EINVAL, "x0 has non-finite entries");
    r.x0[i] = x0[i];
  }
  S.q.push_back(r);
  s->queued += 1;
  if (s->cfg.mode == MPPI_SERVE_PLAIN) s->fifo.push_back(slot);
  return MPPI_OK;
}

extern "C" int mppi_server_poll(mppi_server *s, int32_t max, uint64_t *ids, double *u0s, int32_t *status,
                                double *t_done, int32_t *n) {
  int rc = check_srv(s);
  if (rc) return rc;
  if (!n || max < 0 || (max > 0 && (!ids || !u0s || !status || !t_done))) return fail(MPPI_EINVAL, "bad poll arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  rc = progress(s);
  if (rc) return rc;
  const int k = std::min<int>(max, (int)s->done.size());
  for (int i = 0; i < k; ++i) {
    const Result &r = s->done[i];
    ids[i] = r.id;
    for (int j = 0; j < 4; ++j) u0s[4 * i + j] = r.u0[j];
    status[i] = r.status;
    t_done[i] = r.t_done;
  }
  s->done.erase(s->done.begin(), s->done.begin() + k);
  *n = k;
  return MPPI_OK;
}

extern "C" int mppi_server_replay(mppi_server *s, int32_t n, const double *t_arrival, const int32_t *slots,
                                  const double *x0s, double *t_done, double *u0s, int32_t *status) {
  int rc = check_srv(s);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!t_arrival || !slots || !x0s || !t_done || !u0s || !status)))
    return fail(MPPI_EINVAL, "bad replay arguments");
  for (int i = 1; i < n; ++i)
    if (t_arrival[i] < t_arrival[i - 1]) return fail(MPPI_EINVAL, "arrival times must be non-decreasing");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int i = 0; i < n; ++i)
      if (slots[i] < 0 || slots[i] >= (int)s->slots.size() || !s->slots[slots[i]].used)
        return fail(MPPI_ENOTFOUND, "unknown slot %d", slots[i]);
  }
  const double base = s->now();
  int next = 0, finished = 0;
  std::vector<uint64_t> ids(256);
  std::vector<double> u(4 * 256), td(256);
  std::vector<int32_t> st(256);
  while (finished < n) {
    const double t = s->now() - base;
    while (next < n && t_arrival[next] <= t) {
      rc = mppi_server_submit(s, slots[next], x0s + 16 * (size_t)next, (uint64_t)next, base + t_arrival[next]);
      if (rc) return rc;
      ++next;
    }
    int32_t got = 0;
    rc = mppi_server_poll(s, 256, ids.data(), u.data(), st.data(), td.data(), &got);
    if (rc) return rc;
    for (int i = 0; i < got; ++i) {
      const uint64_t id = ids[i];
      t_done[id] = td[i] - base;
      for (int j = 0; j < 4; ++j) u0s[4 * id + j] = u[4 * i + j];
      status[id] = st[i];
      ++finished;
    }
    if (got == 0 && next < n && t_arrival[next] - (s->now() - base) > 200e-6)
      std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  return MPPI_OK;
}

extern "C" int mppi_server_stats_get(mppi_server *s, mppi_server_stats *o) {
  int rc = check_srv(s);
  if (rc) return rc;
  if (!o) return fail(MPPI_EINVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  o->bytes_used = s->used;
  o->slots_used = 0;
  for (auto &S : s->slots) o->slots_used += S.used ? 1 : 0;
  o->queued = s->queued;
  o->inflight = s->inflight;
  o->requests_done = s->n_done;
  o->batches = s->n_batches;
  o->mean_batch = s->n_batches ? (double)s->n_batched_req / (double)s->n_batches : 0.0;
  o->rollout_steps_done = s->steps_done;
  return MPPI_OK;
}

extern "C" int mppi_server_get_controls(mppi_server *s, int32_t slot, double *u, uint64_t len) {
  int rc = check_srv(s);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  if (slot < 0 || slot >= (int)s->slots.size() || !s->slots[slot].used) return fail(MPPI_ENOTFOUND, "unknown slot %d", slot);
  Slot &S = s->slots[slot];
  if (S.busy) return fail(MPPI_EBUSY, "slot %d has a step in flight", slot);
  return mppi_get_controls(S.ctx, u, len);
}

extern "C" double mppi_server_now(mppi_server *s) { return s ? s->now() : 0.0; }

// Sessions: controllers that arrive, wait for a slot and budget, run, and leave.
extern "C" int mppi_server_replay_sessions(mppi_server *s, int32_t n_sessions, const mppi_config *cfgs,
                                           const double *t_start, const double *t_end, int32_t n,
                                           const double *t_arrival, const int32_t *sessions, const double *x0s,
                                           double *t_done, double *u0s, int32_t *status, double *t_admit,
                                           double *t_release) {
  int rc = check_srv(s);
  if (rc) return rc;
  if (n_sessions < 0 || n < 0 || (n_sessions > 0 && (!cfgs || !t_start || !t_end || !t_admit || !t_release)) ||
      (n > 0 && (!t_arrival || !sessions || !x0s || !t_done || !u0s || !status)))
    return fail(MPPI_EINVAL, "bad replay_sessions arguments");
  std::vector<uint64_t> need(n_sessions);
  for (int j = 0; j < n_sessions; ++j) {
    if (!(t_end[j] >= t_start[j])) return fail(MPPI_EINVAL, "session %d ends before it starts", j);
    rc = mppi_workspace_bytes(&cfgs[j], &need[j]);
    if (rc) return rc;
    t_admit[j] = t_release[j] = -1.0;
  }
  for (int i = 0; i < n; ++i) {
    const int j = sessions[i];
    if (j < 0 || j >= n_sessions) return fail(MPPI_EINVAL, "request %d names session %d of %d", i, j, n_sessions);
    if (t_arrival[i] < t_start[j] || t_arrival[i] >= t_end[j])
      return fail(MPPI_EINVAL, "request %d arrives outside its session's lifetime", i);
    if (i > 0 && t_arrival[i] < t_arrival[i - 1]) return fail(MPPI_EINVAL, "arrival times must be non-decreasing");
  }
  enum { kNotYet, kQueued, kAdmitted, kReleased, kNever };
  std::vector<int> state(n_sessions, kNotYet), slot_of(n_sessions, -1), outstanding(n_sessions, 0);
  std::vector<std::deque<int>> pending(n_sessions);
  std::vector<int> order(n_sessions);
  for (int j = 0; j < n_sessions; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return t_start[a] < t_start[b]; });
  std::deque<int> adm_q;
  std::vector<int> live;                       // admitted sessions
  const double base = s->now();
  int next_s = 0, next_r = 0, finished = 0, done_sessions = 0;
  std::vector<uint64_t> ids(256);
  std::vector<double> u(4 * 256), td(256);
  std::vector<int32_t> st(256);
  auto submit = [&](int i) {
    const int j = sessions[i];
    outstanding[j] += 1;
    return mppi_server_submit(s, slot_of[j], x0s + 16 * (size_t)i, (uint64_t)i, base + t_arrival[i]);
  };
  while (finished < n || done_sessions < n_sessions) {
    const double t = s->now() - base;
    bool acted = false;
    // sessions arriving
    while (next_s < n_sessions && t_start[order[next_s]] <= t) {
      const int j = order[next_s++];
      if (need[j] > s->cfg.hbm_budget_bytes) { state[j] = kNever; ++done_sessions; }
      else { state[j] = kQueued; adm_q.push_back(j); }
      acted = true;
    }
    // admission, first come first served
    while (!adm_q.empty()) {
      const int j = adm_q.front();
      int32_t slot = -1;
      rc = mppi_server_admit(s, &cfgs[j], &slot);
      if (rc == MPPI_EBUSY) break;
      if (rc) return rc;
      adm_q.pop_front();
      state[j] = kAdmitted;
      slot_of[j] = slot;
      t_admit[j] = s->now() - base;
      live.push_back(j);
      while (!pending[j].empty()) {
        rc = submit(pending[j].front());
        if (rc) return rc;
        pending[j].pop_front();
      }
      acted = true;
    }
    // requests arriving
    while (next_r < n && t_arrival[next_r] <= t) {
      const int i = next_r++, j = sessions[i];
      if (state[j] == kAdmitted) {
        rc = submit(i);
        if (rc) return rc;
      } else if (state[j] == kNever) {
        t_done[i] = t_arrival[i];
        for (int q = 0; q < 4; ++q) u0s[4 * (size_t)i + q] = 0.0;
        status[i] = MPPI_EBUSY;
        ++finished;
      } else {
        pending[j].push_back(i);
      }
      acted = true;
    }
    int32_t got = 0;
    rc = mppi_server_poll(s, 256, ids.data(), u.data(), st.data(), td.data(), &got);
    if (rc) return rc;
    for (int q = 0; q < got; ++q) {
      const uint64_t i = ids[q];
      t_done[i] = td[q] - base;
      for (int c = 0; c < 4; ++c) u0s[4 * i + c] = u[4 * q + c];
      status[i] = st[q];
      outstanding[sessions[i]] -= 1;
      ++finished;
    }
    // sessions leaving: past their end (or past the last request of the trace), served
    const bool trace_over = next_r == n;
    for (size_t q = 0; q < live.size();) {
      const int j = live[q];
      if ((t >= t_end[j] || trace_over) && outstanding[j] == 0 && pending[j].empty()) {
        rc = mppi_server_release(s, slot_of[j]);
        if (rc) return rc;
        state[j] = kReleased;
        t_release[j] = s->now() - base;
        ++done_sessions;
        live[q] = live.back();
        live.pop_back();
        acted = true;
      } else {
        ++q;
      }
    }
    if (trace_over && next_s == n_sessions && live.empty() && adm_q.empty()) break;
    if (!acted && got == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  return MPPI_OK;
}
