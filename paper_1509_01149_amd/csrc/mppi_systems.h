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
  // One FP32 Euler step x <- x + dt xdot(x, f) of the rollout, with dt folded into the
  // constants (dt / m, dt g, dt / J_i) so the products by dt merge into the update FMAs.
  // The attitude's sines and cosines take the revolution x / 2 pi straight to the hardware
  // sin / cos, which reduce it themselves (|x| up to 1608 rad; for |x| < pi the argument
  // is the one `rev` forms, bit for bit).  The crash indicator's rollout keeps xdot and a
  // separate update (a crashed sample does not move).
  static constexpr bool kFoldedEuler = true;
  __device__ static void sincos_rev(float x, float &s, float &c) {
    const float r = x * 0.159154943091895335769f;
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
  }
  __device__ static void euler(const Params &p, float *x, const float *f, float dt) {
    float sr, cr, sp, cp, sy, cy;
    sincos_rev(x[6], sr, cr);
    sincos_rev(x[7], sp, cp);
    sincos_rev(x[8], sy, cy);
    const float icp = frcp(cp);
    const float ad = (f[0] + f[1] + f[2] + f[3]) * p.dt_m_inv;
    const float wx = x[9], wy = x[10], wz = x[11];
    const float tx = p.arm * (f[1] - f[3]);
    const float ty = p.arm * (f[2] - f[0]);
    const float tz = p.kap * (f[0] - f[1] + f[2] - f[3]);
    const float hx = p.J[0] * wx, hy = p.J[1] * wy, hz = p.J[2] * wz;
    const float tp = sp * icp;
    // position with the old velocity, velocity with the old attitude, attitude with the old
    // body rates, body rates last
    x[0] = fmaf(dt, x[3], x[0]);
    x[1] = fmaf(dt, x[4], x[1]);
    x[2] = fmaf(dt, x[5], x[2]);
    x[3] = fmaf(ad, cy * sp * cr + sy * sr, x[3]);
    x[4] = fmaf(ad, sy * sp * cr - cy * sr, x[4]);
    x[5] = fmaf(ad, cp * cr, x[5]) - p.dt_g;
    x[6] = fmaf(dt, wx + sr * tp * wy + cr * tp * wz, x[6]);
    x[7] = fmaf(dt, cr * wy - sr * wz, x[7]);
    x[8] = fmaf(dt, (sr * wy + cr * wz) * icp, x[8]);
    x[9] = fmaf(fmaf(wz, hy, fmaf(-wy, hz, tx)), p.dt_Jinv[0], x[9]);
    x[10] = fmaf(fmaf(wx, hz, fmaf(-wz, hx, ty)), p.dt_Jinv[1], x[10]);
    x[11] = fmaf(fmaf(wy, hx, fmaf(-wx, hy, tz)), p.dt_Jinv[2], x[11]);
  }
  // LDS: the obstacles' float4s, then (crash indicator on) their crash thresholds
  static constexpr int stage_floats(int n_obs, int) { return 5 * n_obs; }
  __device__ static void stage(const Params &p, float *lds, const double *, int *, int *) {
    for (int e = threadIdx.x; e < p.n_obs; e += kBlock) reinterpret_cast<float4 *>(lds)[e] = p.obs[e];
    if (p.crash > 0.f) {
      const float *th = reinterpret_cast<const float *>(p.obs + p.n_obs);
      for (int e = threadIdx.x; e < p.n_obs; e += kBlock) lds[4 * p.n_obs + e] = th[e];
    }
  }
  // (r + margin)^2 - |p - c|^2 of obstacle o at position x with xx = |x|^2
  __device__ __forceinline__ static float barrier_arg(const float4 &o, const float *x, float xx) {
    return fmaf(x[0], o.x, fmaf(x[1], o.y, fmaf(x[2], o.z, o.w))) - xx;
  }
  // The obstacles a lane visits first (j, j + nj, ... for kRegObs of them) are held in
  // registers for the whole rollout, the rest are read from LDS each step: with one wave
  // per SIMD, an LDS round trip per obstacle per step would dominate the step.  Unused
  // register slots hold a zero obstacle (argument -|p|^2 <= 0: no barrier, no hit).
  static constexpr int kRegObs = 8;
  struct Regs {
    float4 o[kRegObs];
    float th[kRegObs];
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
  }
  // Lane j of nj: the goal term (j = 0) plus the barriers of obstacles j, j + nj, ...; with
  // kHit also the count of crash conditions among the same obstacles (and the ground for
  // j = 0), from the same barrier arguments.
  template <bool kHit>
  __device__ static float cost_part(const Params &p, const StageView &sv, const Regs &rg, const float *x, int j,
                                    int nj, float &hit) {
    const float dx = x[0] - p.goal[0], dy = x[1] - p.goal[1], dz = x[2] - p.goal[2];
    const float c = j == 0 ? p.wg * (dx * dx + dy * dy + dz * dz) : 0.f;
    const float xx = fmaf(x[0], x[0], fmaf(x[1], x[1], x[2] * x[2]));
    float barrier = 0.f, h = (kHit && j == 0 && x[2] < p.ground) ? 1.f : 0.f;
#pragma unroll
    for (int t = 0; t < kRegObs; ++t) {
      const float arg = barrier_arg(rg.o[t], x, xx);
      const float pen = fmaxf(0.f, arg);
      barrier = fmaf(pen, pen, barrier);
      if (kHit) h += arg > rg.th[t] ? 1.f : 0.f;
    }
    const float4 *ob = reinterpret_cast<const float4 *>(sv.lds);
    const float *th = sv.lds + 4 * p.n_obs;
    // block-uniform: skipped when all fit in registers (the per-lane bounds are formed
    // inside the branch only)
    if (__builtin_expect(p.n_obs > nj * kRegObs, 0)) {
      for (int o = j + nj * kRegObs; o < p.n_obs; o += nj) {
        const float arg = barrier_arg(ob[o], x, xx);
        const float pen = fmaxf(0.f, arg);
        barrier = fmaf(pen, pen, barrier);
        if (kHit) h += arg > th[o] ? 1.f : 0.f;
      }
    }
    hit = h;
    return c + p.wo * barrier;
  }
  static constexpr bool kCrash = true;
  __device__ static float q_part_crash(const Params &p, const StageView &sv, const Regs &rg, const float *x, int j,
                                       int nj, float &hit) {
    return cost_part<true>(p, sv, rg, x, j, nj, hit);
  }
  static constexpr bool kSplitCost = true;
  static constexpr int kLPS = MPPI_ROLLOUT_LPS;
  __device__ static float q_part(const Params &p, const StageView &sv, const Regs &rg, const float *x, int j, int nj) {
    float unused;
    return cost_part<false>(p, sv, rg, x, j, nj, unused);
  }
  __device__ static float q(const Params &p, const StageView &sv, const float *x) {
    const float dx = x[0] - p.goal[0], dy = x[1] - p.goal[1], dz = x[2] - p.goal[2];
    const float c = p.wg * (dx * dx + dy * dy + dz * dz);
    const float xx = fmaf(x[0], x[0], fmaf(x[1], x[1], x[2] * x[2]));
    const float4 *ob = reinterpret_cast<const float4 *>(sv.lds);
    float barrier = 0.f;
    for (int j = 0; j < p.n_obs; ++j) {
      const float pen = fmaxf(0.f, barrier_arg(ob[j], x, xx));
      barrier = fmaf(pen, pen, barrier);
    }
    return c + p.wo * barrier;
  }
  __device__ static float phi(const Params &, const float *) { return 0.f; }
};

}  // namespace mppi
