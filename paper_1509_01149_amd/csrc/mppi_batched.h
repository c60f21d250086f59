// Batched serving kernels: one launch covers the blocks of many controllers.  Each
// controller's per-iteration arguments live in a device-resident descriptor written at
// admission; a per-batch work list names the controllers, their staged start states and
// their result slots.  Every block resolves (controller, local block) from prefix sums
// and runs the same body as the single-controller kernels.
#pragma once
#include "mppi_kernels.h"

namespace mppi {

union SysParams {
  LinearParams lin;
  CartPoleSys::Params cp;
  SwingUpSys::Params su;
  BicycleSys::Params bc;
  QuadrotorSys::Params qd;
};

template <class Sys> __device__ __host__ inline const typename Sys::Params &sys_params(const SysParams &u);
template <> __device__ __host__ inline const LinearParams &sys_params<LinearSys<1>>(const SysParams &u) { return u.lin; }
template <> __device__ __host__ inline const LinearParams &sys_params<LinearSys<2>>(const SysParams &u) { return u.lin; }
template <> __device__ __host__ inline const LinearParams &sys_params<LinearSys<4>>(const SysParams &u) { return u.lin; }
template <> __device__ __host__ inline const CartPoleSys::Params &sys_params<CartPoleSys>(const SysParams &u) { return u.cp; }
template <> __device__ __host__ inline const SwingUpSys::Params &sys_params<SwingUpSys>(const SysParams &u) { return u.su; }
template <> __device__ __host__ inline const BicycleSys::Params &sys_params<BicycleSys>(const SysParams &u) { return u.bc; }
template <> __device__ __host__ inline const QuadrotorSys::Params &sys_params<QuadrotorSys>(const SysParams &u) { return u.qd; }

struct CtrlDesc {
  IterArgs it;          // it.x0 unused: the start state comes from the work item
  FinalizeArgs fin;     // fin.u0_out unused; fin.emit = 1 (one iteration per served step)
  SysParams p;
};

struct WorkItem {
  int desc;             // controller slot
  int pad;
  const double *x0;     // staged start state (device)
  double *out;          // result slot (device): u0[0..3], status at [4]
};

// Largest j with prefix[j] <= b (prefix[0] = 0, strictly increasing over non-empty items).
__device__ __forceinline__ int find_item(const int *__restrict__ prefix, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

template <class Sys, int LPS, int Mode>
__global__ __launch_bounds__(kBlock) void rollout_batched(const CtrlDesc *__restrict__ descs,
                                                          const WorkItem *__restrict__ items,
                                                          const int *__restrict__ sel,
                                                          const int *__restrict__ prefix, int n) {
  extern __shared__ float4 lds4[];
  const int j = find_item(prefix, n, blockIdx.x);
  const WorkItem &w = items[sel[j]];
  const CtrlDesc &d = descs[w.desc];
  // block-uniform copies: the per-step constants live in SGPRs instead of being re-read
  // from the descriptor
  const IterArgs a = d.it;
  const typename Sys::Params p = sys_params<Sys>(d.p);
  const int lb = blockIdx.x - prefix[j];
  if (a.Ushadow && lb == a.n_roll_blocks) {           // the controller's shadow block
    shadow_block<Sys>(a, p);
    return;
  }
  rollout_any<Sys, LPS, Mode>(a, p, w.x0, lb, lds4);
}

static __global__ __launch_bounds__(kBlock) void update_batched(const CtrlDesc *__restrict__ descs,
                                                                const WorkItem *__restrict__ items,
                                                                const int *__restrict__ prefix, int n) {
  if ((int)blockIdx.x >= prefix[n]) return;           // the one-block grid of a batch with no update
  const int j = find_item(prefix, n, blockIdx.x);
  const CtrlDesc &d = descs[items[j].desc];
  const int l = blockIdx.x - prefix[j];
  update_body(d.it, l % d.it.n_kc, l / d.it.n_kc);
}

// One block per controller, or with the multi-block finalize ceil(ceil(T*m / kFinOut) / 4):
// each 1024-thread block then holds four multi-block finalize blocks (prefix over the items).
static_assert(kFinBlock == 4 * kFinMultiBlock, "four multi-block finalize blocks per batched block");
static __global__ __launch_bounds__(kFinBlock) void finalize_batched(const CtrlDesc *__restrict__ descs,
                                                                     const WorkItem *__restrict__ items,
                                                                     const int *__restrict__ prefix, int n) {
  __shared__ double u0_s[4];
  const int j = find_item(prefix, n, blockIdx.x);
  const WorkItem &w = items[j];
  const FinalizeArgs &f = descs[w.desc].fin;
  if (f.multi) {                                       // path weighting
    const int fb = 4 * (blockIdx.x - prefix[j]) + (int)threadIdx.x / kFinMultiBlock;
    finalize_multi_body<1, 4>(f, fb, w.out, w.out + 4, u0_s, [] {});
  } else {
    finalize_body(f, w.out, w.out + 4, u0_s);
  }
}

}  // namespace mppi
