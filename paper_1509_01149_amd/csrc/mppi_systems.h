// Compiled-in systems: dynamics x' = f(x) + G(x) u and state costs q, phi of the
// problem statement (Section II of the paper), one struct per system.  Dynamics are
// templated on the scalar type: FP32 in the rollouts, FP64 in the harness plant.
// The costs run in FP32 inside the rollout and may read system data staged in LDS.
#pragma once
#include "mppi_device.h"

// Lanes per sample of the four-lane rollout body (1 or 4; the quadrotor's); a build-time
// tuning knob.  The step-split systems choose theirs per controller.
#ifndef MPPI_ROLLOUT_LPS
#define MPPI_ROLLOUT_LPS 4
#endif

namespace mppi {

// LDS view handed to a system's cost: its staged data (map tile, obstacles).
struct StageView {
  const float *lds;      // system region of the block's LDS
  int i0, j0;            // bicycle: origin cell of the staged map tile
};

// ------------------------------------------------------------------- linear (tests)
struct LinearParams {
  int n;
  float A[16], B[16], Q[16], Qf[16];   // row-major, leading dimension 4 (B: M)
  double Ad[16], Bd[16];
};
template <int M_>
struct LinearSys {
  static constexpr int N = 4, M = M_;
  using Params = LinearParams;
  template <typename F>
  __device__ static void xdot(const Params &p, const F *x, const F *v, F *xd) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      F s = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) s += (sizeof(F) == 8 ? (F)p.Ad[r * 4 + c] : (F)p.A[r * 4 + c]) * x[c];
#pragma unroll
      for (int c = 0; c < M; ++c) s += (sizeof(F) == 8 ? (F)p.Bd[r * M + c] : (F)p.B[r * M + c]) * v[c];
      xd[r] = s;
    }
  }
  __device__ static float quad(const float *W, const float *x) {
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      float t = 0.f;
#pragma unroll
      for (int c = 0; c < N; ++c) t += W[r * 4 + c] * x[c];
      s += x[r] * t;
    }
    return s;
  }
  // step-split rollout: the cost reads the whole state
  static constexpr bool kStepSplit = true, kOwnChunk = false, kLanes32 = false;
  static constexpr int NQ = N;
  __device__ static void cost_state(const float *x, float *xq) {
#pragma unroll
    for (int r = 0; r < N; ++r) xq[r] = x[r];
  }
  __device__ static float q_step(const Params &p, const float *xq) { return quad(p.Q, xq); }
  __device__ static float q(const Params &p, const StageView &, const float *x) { return quad(p.Q, x); }
  __device__ static float phi(const Params &p, const float *x) { return quad(p.Qf, x); }
};

// ------------------------------------------------------------------------ cart-pole
struct CartPoleSys {
  static constexpr int N = 4, M = 1;
  struct Params {
    float mc, mp, l, g, qd[4], qfd[4];
    double dmc, dmp, dl, dg;
  };
  template <typename F>
  __device__ static void xdot(const Params &p, const F *x, const F *v, F *xd) {
    const bool d = sizeof(F) == 8;
    const F mc = d ? (F)p.dmc : (F)p.mc, mp = d ? (F)p.dmp : (F)p.mp;
    const F l = d ? (F)p.dl : (F)p.l, g = d ? (F)p.dg : (F)p.g;
    const F Mt = mc + mp;
    const F iM = frcp(Mt);
    F s, c;
    fsincos(x[2], s, c);
    const F h = (v[0] + mp * l * x[3] * x[3] * s) * iM;
    const F thdd = (g * s - c * h) * frcp(l * ((F)(4.0 / 3.0) - mp * c * c * iM));
    xd[0] = x[1];
    xd[1] = h - mp * l * thdd * c * iM;
    xd[2] = x[3];
    xd[3] = thdd;
  }
  __device__ static float q(const Params &p, const StageView &, const float *x) {
    return p.qd[0] * x[0] * x[0] + p.qd[1] * x[1] * x[1] + p.qd[2] * x[2] * x[2] + p.qd[3] * x[3] * x[3];
  }
  static constexpr bool kStepSplit = true, kOwnChunk = true, kLanes32 = false;
  static constexpr int NQ = N;
  __device__ static void cost_state(const float *x, float *xq) {
#pragma unroll
    for (int r = 0; r < N; ++r) xq[r] = x[r];
  }
  __device__ static float q_step(const Params &p, const float *xq) { return q(p, StageView{}, xq); }
  __device__ static float phi(const Params &p, const float *x) {
    return p.qfd[0] * x[0] * x[0] + p.qfd[1] * x[1] * x[1] + p.qfd[2] * x[2] * x[2] + p.qfd[3] * x[3] * x[3];
  }
  // One chunk of the step-split rollout.  The pole's angle and rate do not depend on the
  // cart's position or velocity, so every lane steps only the pole through the chunk (the
  // FP32 expressions of xdot), with the owners' forces broadcast, and keeps the cart
  // acceleration of its own steps and the pole state after them; the cart's velocity
  // (adding dt xddot) and position (adding dt times the velocity before the step) are
  // then prefix sums over the chunk.  Steps past the horizon leave the state unchanged.
  // du: this lane's perturbations (SPG steps); xq: state after its steps.
  template <int LPS, int SPG, bool kChecked>
  __device__ static void chunk(const Params &p, int T, float dt, const float *sU, const float *du, int g0,
                               int lane_j, float *x, float (*xq)[NQ]) {
    const int i_first = (g0 + lane_j) * SPG;
    bool ok[SPG];
    float f[SPG];                                  // own steps: applied force
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      const int i = i_first + s;
      ok[s] = !kChecked || i < T;
      f[s] = sU[min(i, T - 1)] + du[s];
    }
    const float mc = p.mc, mp = p.mp, l = p.l, g = p.g;
    const float Mt = mc + mp;
    const float iM = frcp(Mt);
    float xa[SPG], th[SPG], om[SPG];               // own steps: cart acceleration, pole after
#pragma unroll
    for (int s = 0; s < SPG; ++s) xa[s] = th[s] = om[s] = 0.f;
    StaticFor<0, LPS>::run([&](auto jc) {
      constexpr int JJ = decltype(jc)::value;
      const int i0 = (g0 + JJ) * SPG;
      if (!kChecked || i0 < T) {
        float fj[SPG];
#pragma unroll
        for (int s = 0; s < SPG; ++s) fj[s] = group_bcast<LPS, JJ>(f[s]);
        const bool mine = lane_j == JJ;
#pragma unroll
        for (int s = 0; s < SPG; ++s) {
          if (!kChecked || i0 + s < T) {
            float sn, cs;
            fsincos(x[2], sn, cs);
            const float h = (fj[s] + mp * l * x[3] * x[3] * sn) * iM;
            const float thdd = (g * sn - cs * h) * frcp(l * ((float)(4.0 / 3.0) - mp * cs * cs * iM));
            const float xdd = h - mp * l * thdd * cs * iM;
            x[2] += dt * x[3];
            x[3] += dt * thdd;
            xa[s] = mine ? xdd : xa[s];
            th[s] = mine ? x[2] : th[s];
            om[s] = mine ? x[3] : om[s];
            // keep each capture at its step: sunk to the chunk's end, the selects would hold
            // every step's candidates live (about three times the registers)
            asm volatile("" : "+v"(xa[s]), "+v"(th[s]), "+v"(om[s]));
          }
        }
      }
    });
    // cart velocity, then position: running sums across the group
    float inc[SPG], own = 0.f;
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      inc[s] = ok[s] ? dt * xa[s] : 0.f;
      own += inc[s];
    }
    float w = x[1] + group_excl_of_incl<LPS>(group_scan_incl<LPS>(own, lane_j), lane_j);
    float vb[SPG], va[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      vb[s] = w;
      w += inc[s];
      va[s] = w;
    }
    x[1] = group_bcast<LPS, LPS - 1>(w);
    float pinc[SPG], pown = 0.f;
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      pinc[s] = ok[s] ? dt * vb[s] : 0.f;
      pown += pinc[s];
    }
    float r = x[0] + group_excl_of_incl<LPS>(group_scan_incl<LPS>(pown, lane_j), lane_j);
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      r += pinc[s];
      xq[s][0] = r;
      xq[s][1] = va[s];
      xq[s][2] = th[s];
      xq[s][3] = om[s];
    }
    x[0] = group_bcast<LPS, LPS - 1>(r);
  }
};

// ------------------------------------------------ cart-pole swing-up (velocity command)
// The cart tracks the commanded velocity through pddot = gain (u - pdot); the pole turns
// about the accelerated pivot, theta = 0 hanging down.
struct SwingUpSys {
  static constexpr int N = 4, M = 1;
  struct Params {
    float gain, k, g, wp, wa, wv, wr;    // k = 3 / (4 l)
    double dgain, dk, dg;
  };
  template <typename F>
  __device__ static void xdot(const Params &p, const F *x, const F *v, F *xd) {
    const bool d = sizeof(F) == 8;
    const F gain = d ? (F)p.dgain : (F)p.gain, k = d ? (F)p.dk : (F)p.k, g = d ? (F)p.dg : (F)p.g;
    const F pdd = gain * (v[0] - x[1]);
    xd[0] = x[1];
    xd[1] = pdd;
    xd[2] = x[3];
    F s, c;
    fsincos(x[2], s, c);
    xd[3] = -k * (g * s + pdd * c);
  }
  __device__ static float q(const Params &p, const StageView &, const float *x) {
    const float a = 1.f + fcos(x[2]);
    return p.wp * x[0] * x[0] + p.wa * a * a + p.wr * x[3] * x[3] + p.wv * x[1] * x[1];
  }
  static constexpr bool kStepSplit = true, kOwnChunk = true, kLanes32 = false;   // affine scans: 4 or 16
  static constexpr int NQ = N;
  __device__ static void cost_state(const float *x, float *xq) {
#pragma unroll
    for (int r = 0; r < N; ++r) xq[r] = x[r];
  }
  __device__ static float q_step(const Params &p, const float *xq) { return q(p, StageView{}, xq); }
  __device__ static float phi(const Params &, const float *) { return 0.f; }
  // One chunk of the step-split rollout.  The cart is driven by the command alone: its
  // velocity follows the affine map pdot -> (1 - dt gain) pdot + dt gain u and its
  // position adds dt pdot, so both are prefix scans over the chunk (the velocity's a scan
  // of affine maps); each lane then forms the cart acceleration of its own steps, and the
  // pole's angle and rate, the only part with a per-step chain, are stepped in every lane
  // with those accelerations broadcast from their owners.  Steps past the horizon leave
  // the state unchanged.  du: this lane's perturbations (SPG steps); xq: state after its
  // steps.
  template <int LPS, int SPG, bool kChecked>
  __device__ static void chunk(const Params &p, int T, float dt, const float *sU, const float *du, int g0,
                               int lane_j, float *x, float (*xq)[NQ]) {
    const int i_first = (g0 + lane_j) * SPG;
    const float ca = 1.f - dt * p.gain, cb = dt * p.gain;
    bool ok[SPG];
    float v[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      const int i = i_first + s;
      ok[s] = !kChecked || i < T;
      v[s] = sU[min(i, T - 1)] + du[s];
    }
    // cart velocity: this lane's composed map, the maps before it, then its own steps
    float A = 1.f, B = 0.f;
#pragma unroll
    for (int s = 0; s < SPG; ++s)
      if (ok[s]) {
        B = fmaf(ca, B, cb * v[s]);
        A = ca * A;
      }
    group_affine_scan_incl<LPS>(A, B, lane_j);
    group_affine_excl_of_incl<LPS>(A, B, lane_j);
    float w = fmaf(A, x[1], B);                     // cart velocity before this lane's steps
    float vb[SPG], va[SPG], pdd[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      vb[s] = w;
      pdd[s] = p.gain * (v[s] - w);
      if (ok[s]) w = fmaf(ca, w, cb * v[s]);
      va[s] = w;
    }
    x[1] = group_bcast<LPS, LPS - 1>(w);
    // cart position: running sum of dt pdot
    float own = 0.f, inc[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      inc[s] = ok[s] ? dt * vb[s] : 0.f;
      own += inc[s];
    }
    float r = x[0] + group_excl_of_incl<LPS>(group_scan_incl<LPS>(own, lane_j), lane_j);
    float pa[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      r += inc[s];
      pa[s] = r;
    }
    x[0] = group_bcast<LPS, LPS - 1>(r);
    // pole: every lane steps angle and rate through the chunk
    float th[SPG], om[SPG];
#pragma unroll
    for (int s = 0; s < SPG; ++s) th[s] = om[s] = 0.f;
    StaticFor<0, LPS>::run([&](auto jc) {
      constexpr int JJ = decltype(jc)::value;
      const int i0 = (g0 + JJ) * SPG;
      if (!kChecked || i0 < T) {
        float a_c[SPG];
#pragma unroll
        for (int s = 0; s < SPG; ++s) a_c[s] = group_bcast<LPS, JJ>(pdd[s]);
        const bool mine = lane_j == JJ;
#pragma unroll
        for (int s = 0; s < SPG; ++s) {
          if (!kChecked || i0 + s < T) {
            float sn, cs;
            fsincos(x[2], sn, cs);
            const float al = -p.k * (p.g * sn + a_c[s] * cs);
            x[2] += dt * x[3];
            x[3] += dt * al;
            th[s] = mine ? x[2] : th[s];
            om[s] = mine ? x[3] : om[s];
          }
        }
      }
    });
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      xq[s][0] = pa[s];
      xq[s][1] = va[s];
      xq[s][2] = th[s];
      xq[s][3] = om[s];
    }
  }
};

// ------------------------------------------------------------ kinematic bicycle + map
// The cost map (FP32, [y][x]) stays in HBM; the step-split rollout evaluates each step's
// cost a chunk after the state is known and reads the bilinear taps from global memory
// (the map stays resident in L2).
struct BicycleSys {
  static constexpr int N = 5, M = 2;
  struct Params {
    float L_inv, vt, ws, cell_inv, lim;
    int W, H;
    const float *map;                 // device
    double dL_inv, dlim;
  };
  template <typename F>
  __device__ static void xdot(const Params &p, const F *x, const F *v, F *xd) {
    const bool d = sizeof(F) == 8;
    const F lim = d ? (F)p.dlim : (F)p.lim;
    F dl = x[4];
    if (lim > 0) dl = dl < -lim ? -lim : (dl > lim ? lim : dl);
    F s, c, sd, cd;
    fsincos(x[2], s, c);
    fsincos(dl, sd, cd);
    const F tn = sd * frcp(cd);
    xd[0] = x[3] * c;
    xd[1] = x[3] * s;
    xd[2] = x[3] * tn * (d ? (F)p.dL_inv : (F)p.L_inv);
    xd[3] = v[0];
    xd[4] = v[1];
  }
  // Step-split rollout: the cost needs position and speed only, and reads the bilinear
  // taps straight from the map in global memory (L2-resident; no LDS window, so no
  // fallback).  Same arithmetic and tap values as q().
  static constexpr bool kStepSplit = true, kOwnChunk = true, kLanes32 = true;
  static constexpr int NQ = 3;
  __device__ static void cost_state(const float *x, float *xq) { xq[0] = x[0]; xq[1] = x[1]; xq[2] = x[3]; }
  // One chunk of the step-split rollout.  Every state update of the bicycle is a running
  // sum once its increment is known: speed and steering add dt times the controls, heading
  // adds dt x3 tan(d)/L, position adds dt x3 (cos, sin)(heading).  So each is a prefix sum
  // over the chunk's steps: a lane adds the increments of its own steps, a DPP scan over
  // the lane group gives every lane the value at the start of its steps, and the group's
  // last lane holds the value at the end of the chunk.  Three rounds (speed and steering,
  // heading, position), each preceded by the increments of the lane's own steps (the only
  // transcendentals: once per step).  Steps past the horizon add nothing.
  // du: this lane's group perturbations (SPG steps x M); xq: cost state after its steps.
  template <int LPS, int SPG, bool kChecked>
  __device__ static void chunk(const Params &p, int T, float dt, const float *sU, const float *du, int g0,
                               int lane_j, float *x, float (*xq)[NQ]) {
    const int i_first = (g0 + lane_j) * SPG;
    bool ok[SPG];
    float a3[SPG], a4[SPG];                        // own steps: speed and steering increments
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      const int i = i_first + s;
      ok[s] = !kChecked || i < T;
      const int ic = min(i, T - 1);
      a3[s] = ok[s] ? dt * (sU[ic * M] + du[s * M]) : 0.f;
      a4[s] = ok[s] ? dt * (sU[ic * M + 1] + du[s * M + 1]) : 0.f;
    }
    // running sums of this lane's increments, then the scan across the group
    auto scan = [&](const float *inc, float start, float *before, float *after) {
      float own = inc[0];
#pragma unroll
      for (int s = 1; s < SPG; ++s) own += inc[s];
      float r = start + group_excl_of_incl<LPS>(group_scan_incl<LPS>(own, lane_j), lane_j);
#pragma unroll
      for (int s = 0; s < SPG; ++s) {
        if (before) before[s] = r;
        r += inc[s];
        if (after) after[s] = r;
      }
      return group_bcast<LPS, LPS - 1>(r);         // the value after the chunk
    };
    float vb[SPG], db[SPG], va[SPG];
    x[3] = scan(a3, x[3], vb, va);
    x[4] = scan(a4, x[4], db, nullptr);
    float a2[SPG];                                 // own steps: heading increments
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      float dl = db[s];
      if (p.lim > 0) dl = dl < -p.lim ? -p.lim : (dl > p.lim ? p.lim : dl);
      float sd, cd;
      fsincos(dl, sd, cd);
      const float tn = sd * frcp(cd);
      a2[s] = ok[s] ? dt * (vb[s] * tn * p.L_inv) : 0.f;
    }
    float hb[SPG];
    x[2] = scan(a2, x[2], hb, nullptr);
    float a0[SPG], a1[SPG];                        // own steps: position increments
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      float sn, cs;
      fsincos(hb[s], sn, cs);
      a0[s] = ok[s] ? dt * (vb[s] * cs) : 0.f;
      a1[s] = ok[s] ? dt * (vb[s] * sn) : 0.f;
    }
    float pa0[SPG], pa1[SPG];
    x[0] = scan(a0, x[0], nullptr, pa0);
    x[1] = scan(a1, x[1], nullptr, pa1);
#pragma unroll
    for (int s = 0; s < SPG; ++s) {
      xq[s][0] = pa0[s];
      xq[s][1] = pa1[s];
      xq[s][2] = va[s];
    }
  }
  __device__ static float q_step(const Params &p, const float *xq) {
    float gx = xq[0] * p.cell_inv, gy = xq[1] * p.cell_inv;
    gx = fminf(fmaxf(gx, 0.f), (float)(p.W - 1));
    gy = fminf(fmaxf(gy, 0.f), (float)(p.H - 1));
    const int i0 = min((int)floorf(gx), p.W - 2);
    const int j0 = min((int)floorf(gy), p.H - 2);
    const float fx = gx - (float)i0, fy = gy - (float)j0;
    const __attribute__((address_space(1))) float *g =
        (const __attribute__((address_space(1))) float *)p.map + ((size_t)j0 * p.W + i0);
    const float m00 = g[0], m01 = g[1], m10 = g[p.W], m11 = g[p.W + 1];
    const float top = (1.f - fx) * m00 + fx * m01;
    const float bot = (1.f - fx) * m10 + fx * m11;
    const float dv = xq[2] - p.vt;
    return (1.f - fy) * top + fy * bot + p.ws * dv * dv;
  }
  __device__ static float phi(const Params &, const float *) { return 0.f; }
};

// ------------------------------------------------------------------------ quadrotor
struct QuadrotorSys {
  static constexpr int N = 12, M = 4;
  static constexpr int kMaxObstacles = 256;
  static constexpr bool kStepSplit = false;   // obstacles split over the quad instead
  struct Params {
    float m_inv, g, arm, kap, J[3], Jinv[3], goal[3], wg, wo, margin;
    int n_obs;
    // device: n_obs x (2 c, (r + margin)^2 - |c|^2), then n_obs x ((r + margin)^2 - r^2): the
    // barrier's argument (r + margin)^2 - |p - c|^2 = w + 2 c . p - |p|^2 is three FMAs from
    // |p|^2, and the crash test |p - c| < r is that argument above the second value
    const float4 *obs;
    float crash, ground; // crash indicator cost (0: off) and ground height
    float dt_m_inv, dt_g, dt_Jinv[3];   // dt / m, dt g, dt / J_i (the folded Euler step)
    float dt_rev;                       // dt / (2 pi): the folded step holds the attitude in revolutions
    // The obstacle scale s, a power of two with s (r + margin)^2 <= 1/4 for every obstacle:
    // the device obstacles hold s (2 c, (r + margin)^2 - |c|^2) and s ((r + margin)^2 - r^2),
    // so the barrier argument comes out times s (exactly: s is a power of two) and lies in
    // (-inf, 1/4]; wo_s = w_obs / s^2 restores the barrier's weight.
    float obs_scale, wo_s;
    // The goal term w_g |p - goal|^2 expanded as gq s|p|^2 + glin . p + gconst, with
    // gq = w_g / s, glin = -2 w_g goal, gconst = w_g |goal|^2 (which joins the per-step
    // control cost, so the cost chain starts from the likelihood-ratio terms).
    float gq, glin[3], gconst;
    double dm_inv, dg, darm, dkap, dJ[3], dJinv[3];
  };
  template <typename F>
  __device__ static void xdot(const Params &p, const F *x, const F *f, F *xd) {
    const bool d = sizeof(F) == 8;
    const F m_inv = d ? (F)p.dm_inv : (F)p.m_inv, g = d ? (F)p.dg : (F)p.g;
    const F arm = d ? (F)p.darm : (F)p.arm, kap = d ? (F)p.dkap : (F)p.kap;
    const F J0 = d ? (F)p.dJ[0] : (F)p.J[0], J1 = d ? (F)p.dJ[1] : (F)p.J[1], J2 = d ? (F)p.dJ[2] : (F)p.J[2];
    const F Ji0 = d ? (F)p.dJinv[0] : (F)p.Jinv[0], Ji1 = d ? (F)p.dJinv[1] : (F)p.Jinv[1],
            Ji2 = d ? (F)p.dJinv[2] : (F)p.Jinv[2];
    F sr, cr, sp, cp, sy, cy;
    fsincos(x[6], sr, cr);
    fsincos(x[7], sp, cp);
    fsincos(x[8], sy, cy);
    const F a = (f[0] + f[1] + f[2] + f[3]) * m_inv;
    xd[0] = x[3];
    xd[1] = x[4];
    xd[2] = x[5];
    // third column of R = Rz(yaw) Ry(pitch) Rx(roll)
    xd[3] = a * (cy * sp * cr + sy * sr);
    xd[4] = a * (sy * sp * cr - cy * sr);
    xd[5] = a * (cp * cr) - g;
    const F icp = frcp(cp);
    const F tp = sp * icp;
    const F wx = x[9], wy = x[10], wz = x[11];
    xd[6] = wx + sr * tp * wy + cr * tp * wz;
    xd[7] = cr * wy - sr * wz;
    xd[8] = (sr * wy + cr * wz) * icp;
    const F tx = arm * (f[1] - f[3]);
    const F ty = arm * (f[2] - f[0]);
    const F tz = kap * (f[0] - f[1] + f[2] - f[3]);
    // tau - w x (J w), as explicit FMAs
    const F hx = J0 * wx, hy = J1 * wy, hz = J2 * wz;
    xd[9] = fma(wz, hy, fma(-wy, hz, tx)) * Ji0;
    xd[10] = fma(wx, hz, fma(-wz, hx, ty)) * Ji1;
    xd[11] = fma(wy, hx, fma(-wx, hy, tz)) * Ji2;
  }
  // The rollout's FP32 Euler step x <- x + dt xdot(x, u) with its constants folded:
  //  - dt enters the constants (dt / m, dt g, dt / J_i, dt / 2 pi), so the products by dt
  //    merge into the update FMAs;
  //  - the attitude is held in revolutions (init_state), which the hardware sin / cos take
  //    directly and reduce themselves (|x| up to 256 revolutions);
  //  - the thrusts enter the dynamics only through four linear combinations, the collective
  //    thrust times dt / m and the three body torques; the rollout forms them for the nominal
  //    controls once per step (fold_controls on u_i, staged in LDS) and adds the fold of the
  //    perturbation as a fixed 4 x 4 map of the step's normals (fold_controls on each column
  //    of the noise map A chol(Sigma)).
  // Under the crash indicator a crashed sample skips the step (it does not move).
  static constexpr bool kFoldedEuler = true;
  __device__ static void init_state(const double *x0, int n, float *x) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const double v = r < n ? x0[r] : 0.0;
      x[r] = (float)(r >= 6 && r < 9 ? v * 0.15915494309189533577 : v);
    }
  }
  // (dt / m sum u, arm (u_1 - u_3), arm (u_2 - u_0), kap (u_0 - u_1 + u_2 - u_3))
  __device__ static float4 fold_controls(const Params &p, float u0, float u1, float u2, float u3) {
    return make_float4(((u0 + u1) + (u2 + u3)) * p.dt_m_inv, p.arm * (u1 - u3), p.arm * (u2 - u0),
                       p.kap * ((u0 - u1) + (u2 - u3)));
  }
  // The fold of a step's perturbation from its normals e, W[l] the fold of column l of the
  // noise map.  kDiag: the noise map is diagonal, so the torques about x and y take two
  // normals each (the other two coefficients are exact zeros).
  template <bool kDiag>
  __device__ static float4 fold_noise(const float4 *W, const float *e) {
    float ad = 0.f, tx = 0.f, ty = 0.f, tz = 0.f;
#pragma unroll
    for (int l = 3; l >= 0; --l) {
      ad = fmaf(W[l].x, e[l], ad);
      if (!kDiag || l == 1 || l == 3) tx = fmaf(W[l].y, e[l], tx);
      if (!kDiag || l == 0 || l == 2) ty = fmaf(W[l].z, e[l], ty);
      tz = fmaf(W[l].w, e[l], tz);
    }
    return make_float4(ad, tx, ty, tz);
  }
  // nom: the fold of u_i; nf: the fold of the step's perturbation.
  __device__ static void euler_folded(const Params &p, float dt, float *x, float4 nom, float4 nf) {
    const float ad = nom.x + nf.x, tx = nom.y + nf.y, ty = nom.z + nf.z, tz = nom.w + nf.w;
    const float sr = __builtin_amdgcn_sinf(x[6]), cr = __builtin_amdgcn_cosf(x[6]);
    const float sp = __builtin_amdgcn_sinf(x[7]), cp = __builtin_amdgcn_cosf(x[7]);
    const float sy = __builtin_amdgcn_sinf(x[8]), cy = __builtin_amdgcn_cosf(x[8]);
    const float icp = frcp(cp);
    const float wx = x[9], wy = x[10], wz = x[11];
    const float spcr = sp * cr;
    const float b = fmaf(cr, wz, sr * wy);           // sr wy + cr wz
    const float tp = sp * icp;
    // position with the old velocity, velocity with the old attitude (third column of
    // Rz(yaw) Ry(pitch) Rx(roll)), attitude with the old body rates, body rates last
    x[0] = fmaf(dt, x[3], x[0]);
    x[1] = fmaf(dt, x[4], x[1]);
    x[2] = fmaf(dt, x[5], x[2]);
    x[3] = fmaf(ad, fmaf(cy, spcr, sy * sr), x[3]);
    x[4] = fmaf(ad, fmaf(sy, spcr, -(cy * sr)), x[4]);
    x[5] = fmaf(ad, cp * cr, x[5]) - p.dt_g;
    x[6] = fmaf(p.dt_rev, fmaf(tp, b, wx), x[6]);
    x[7] = fmaf(p.dt_rev, fmaf(cr, wy, -(sr * wz)), x[7]);
    x[8] = fmaf(p.dt_rev, b * icp, x[8]);
    // tau - w x (J w) of a diagonal J: tau_x + (J_y - J_z) w_y w_z and its cyclic shifts
    x[9] = fmaf(fmaf(p.J[1] - p.J[2], wy * wz, tx), p.dt_Jinv[0], x[9]);
    x[10] = fmaf(fmaf(p.J[2] - p.J[0], wz * wx, ty), p.dt_Jinv[1], x[10]);
    x[11] = fmaf(fmaf(p.J[0] - p.J[1], wx * wy, tz), p.dt_Jinv[2], x[11]);
  }
  // LDS: the obstacles' float4s, then (crash indicator on) their crash thresholds
  static constexpr int stage_floats(int n_obs, int) { return 5 * n_obs; }
  __device__ static int staged_floats(const Params &p) { return stage_floats(p.n_obs, 0); }
  __device__ static void stage(const Params &p, float *lds, const double *, int *, int *) {
    for (int e = threadIdx.x; e < p.n_obs; e += kBlock) reinterpret_cast<float4 *>(lds)[e] = p.obs[e];
    if (p.crash > 0.f) {
      const float *th = reinterpret_cast<const float *>(p.obs + p.n_obs);
      for (int e = threadIdx.x; e < p.n_obs; e += kBlock) lds[4 * p.n_obs + e] = th[e];
    }
  }
  // s ((r + margin)^2 - |p - c|^2) of (scaled) obstacle o at position x, with xx = s |x|^2
  __device__ __forceinline__ static float barrier_arg(const float4 &o, const float *x, float xx) {
    return fmaf(x[0], o.x, fmaf(x[1], o.y, fmaf(x[2], o.z, o.w))) - xx;
  }
  // s |x|^2 of a position
  __device__ __forceinline__ static float scaled_sq(const Params &p, const float *x) {
    return fmaf(x[0], x[0], fmaf(x[1], x[1], x[2] * x[2])) * p.obs_scale;
  }
  // The barrier's penalty max(0, arg) of a scaled argument.  The argument is at most 1/4
  // in exact arithmetic, so clamping to [0, 1] gives the same value (a rollout far enough
  // out for rounding to push it past 1 has diverged); the clamp folds into the subtract
  // that forms the argument.
  __device__ __forceinline__ static float penalty(float arg) { return fminf(fmaxf(arg, 0.f), 1.f); }
  // The obstacles a lane visits first (j, j + nj, ... for kRegObs of them) are held in
  // registers for the whole rollout, the rest are read from LDS each step: with one wave
  // per SIMD, an LDS round trip per obstacle per step would dominate the step.  Unused
  // register slots hold a zero obstacle (argument -s|p|^2 <= 0: no barrier, no hit).  The
  // goal term's coefficients sit in lane 0 of the group; the other lanes hold zeros.
  static constexpr int kRegObs = 8;
  struct Regs {
    float4 o[kRegObs];
    float th[kRegObs];
    float gq, glin[3];
  };
  __device__ static void load_regs(const Params &p, const StageView &sv, int j, int nj, Regs &rg) {
    const float4 *ob = reinterpret_cast<const float4 *>(sv.lds);
    const float *th = sv.lds + 4 * p.n_obs;
#pragma unroll
    for (int t = 0; t < kRegObs; ++t) {
      const int o = j + nj * t;
      const bool in = o < p.n_obs;
      rg.o[t] = in ? ob[o] : make_float4(0.f, 0.f, 0.f, 0.f);
      rg.th[t] = in && p.crash > 0.f ? th[o] : 0.f;
    }
    rg.gq = j == 0 ? p.gq : 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) rg.glin[d] = j == 0 ? p.glin[d] : 0.f;
  }
  // The per-step constant of the state cost (the goal term's w_g |goal|^2): the rollout
  // adds it to the per-step control cost u_i'R u_i / 2, which lane 0 carries into `base`.
  static constexpr bool kStepConst = true;
  __device__ static float step_const(const Params &p) { return p.gconst; }
  // Whether lanes of nj-lane groups need the LDS pass (more obstacles than registers hold).
  __device__ static bool lds_pass(const Params &p, int nj) { return p.n_obs > nj * kRegObs; }
  // Lane j of nj: base (this lane's likelihood-ratio share), the goal term (j = 0) and the
  // barriers of obstacles j, j + nj, ...; with kHit also, in `hit`, the largest crash margin
  // among the same obstacles (and the ground for j = 0): max of pen - (the obstacle's
  // threshold) and ground - z, positive exactly when one crash condition holds (the sign of
  // a rounded difference is the sign of the exact one).  pen is the clamped argument, so
  // the clamp still folds into the subtract: a threshold lies in [0, 1/4], so pen - th > 0
  // exactly when arg - th > 0 (equal values for arg in [0, 1]; both negative or zero below
  // 0, both positive above 1).
  template <bool kHit, bool kRegOnly>
  __device__ static float cost_part(const Params &p, const StageView &sv, const Regs &rg, const float *x, int j,
                                    int nj, float base, float &hit) {
    const float xx = scaled_sq(p, x);
    const float c = fmaf(rg.gq, xx, fmaf(x[0], rg.glin[0], fmaf(x[1], rg.glin[1], fmaf(x[2], rg.glin[2], base))));
    float barrier = 0.f, h = 0.f;
    if constexpr (kHit) h = j == 0 ? p.ground - x[2] : -__builtin_inff();
#pragma unroll
    for (int t = 0; t < kRegObs; ++t) {
      const float pen = penalty(barrier_arg(rg.o[t], x, xx));
      barrier = fmaf(pen, pen, barrier);
      if constexpr (kHit) h = fmaxf(h, pen - rg.th[t]);
    }
    const float4 *ob = reinterpret_cast<const float4 *>(sv.lds);
    const float *th = sv.lds + 4 * p.n_obs;
    // block-uniform: skipped when all fit in registers (the per-lane bounds are formed
    // inside the branch only); left out of the code with kRegOnly
    if (!kRegOnly && __builtin_expect(lds_pass(p, nj), 0)) {
      for (int o = j + nj * kRegObs; o < p.n_obs; o += nj) {
        const float pen = penalty(barrier_arg(ob[o], x, xx));
        barrier = fmaf(pen, pen, barrier);
        if constexpr (kHit) h = fmaxf(h, pen - th[o]);
      }
    }
    hit = h;
    return fmaf(p.wo_s, barrier, c);
  }
  static constexpr bool kCrash = true;
  template <bool kRegOnly>
  __device__ static float q_part_crash(const Params &p, const StageView &sv, const Regs &rg, const float *x, int j,
                                       int nj, float base, float &hit) {
    return cost_part<true, kRegOnly>(p, sv, rg, x, j, nj, base, hit);
  }
  static constexpr bool kSplitCost = true;
  static constexpr int kLPS = MPPI_ROLLOUT_LPS;
  template <bool kRegOnly>
  __device__ static float q_part(const Params &p, const StageView &sv, const Regs &rg, const float *x, int j, int nj,
                                 float base) {
    float unused;
    return cost_part<false, kRegOnly>(p, sv, rg, x, j, nj, base, unused);
  }
  // The whole state cost in one lane (less step_const, which the control cost carries).
  __device__ static float q(const Params &p, const StageView &sv, const float *x) {
    const float xx = scaled_sq(p, x);
    const float c = fmaf(p.gq, xx, fmaf(x[0], p.glin[0], fmaf(x[1], p.glin[1], x[2] * p.glin[2])));
    const float4 *ob = reinterpret_cast<const float4 *>(sv.lds);
    float barrier = 0.f;
    for (int j = 0; j < p.n_obs; ++j) {
      const float pen = penalty(barrier_arg(ob[j], x, xx));
      barrier = fmaf(pen, pen, barrier);
    }
    return fmaf(p.wo_s, barrier, c);
  }
  __device__ static float phi(const Params &, const float *) { return 0.f; }
};

}  // namespace mppi
