"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: initial states, the bicycle cost map, the
quadrotor obstacle field, MLP training inputs and serving arrival traces.  It
holds none of the method's arithmetic (no dynamics, no costs, no noise, no
weights) so that the CPU oracle and the HIP path can both consume it without
sharing any code that the parity tests are meant to check.

Random numbers here come from NumPy's PCG64 stream keyed by a fixed seed.  The
rollout noise that MPPI itself draws is *not* generated here: each side
implements Philox4x32-10 on its own.

The paper gives no system constants for its experiments (its race-car tire model
and quadrotor model are cited, not printed), so the systems below are synthetic
stand-ins with the shapes of the paper's three experiments (Section V: cart-pole,
race car, quadrotor in an obstacle field).  Every constant that the paper leaves
open carries a ``# builder-choice`` tag.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

# System identifiers; they match the enum in include/mppi.h.
SYS_LINEAR = 0
SYS_CARTPOLE = 1
SYS_BICYCLE = 2
SYS_QUADROTOR = 3
SYS_QUADROTOR_MLP = 4
SYS_CARTPOLE_SWINGUP = 5
SYSTEM_NAMES = {SYS_LINEAR: "linear", SYS_CARTPOLE: "cartpole", SYS_BICYCLE: "bicycle",
                SYS_QUADROTOR: "quadrotor", SYS_QUADROTOR_MLP: "quadrotor_mlp",
                SYS_CARTPOLE_SWINGUP: "cartpole_swingup"}

# Seeds of the input streams (builder-choice, frozen).
SEED_X0 = 100
SEED_MAP = 7
SEED_OBSTACLES = 11
SEED_MLP_DATA = 3
SEED_MLP_INIT = 5
SEED_SERVING = 12345


@dataclasses.dataclass
class Workload:
    """One MPPI problem: the quantities Algorithm 1 is given (Section IV).

    sigma is the natural per-step covariance of the control perturbation
    (a variance, m x m); nu scales it for exploration (Section III-C, A = sqrt(nu) I);
    R is the per-step control-cost matrix used in the likelihood-ratio cost terms;
    lam is the temperature of the exponential weights.
    """
    name: str
    system: int
    n: int
    m: int
    K: int
    T: int
    dt: float
    sigma: np.ndarray
    nu: float
    lam: float
    R: np.ndarray
    u_init: np.ndarray
    params: Dict
    x0: np.ndarray
    seed: int = 0
    n_iters: int = 1
    control_steps: int = 1

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------- inputs

def uniform_states(n_states: int, lo, hi, seed: int = SEED_X0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n_states, lo.size))


def cost_map(width: int = 256, height: int = 256, n_bumps: int = 40, seed: int = SEED_MAP) -> np.ndarray:
    """256x256 FP32 terrain cost: a sum of seeded isotropic Gaussian bumps.

    Bump centres ~ U[0, 256)^2 cells, widths sigma ~ U[3, 12] cells, heights ~ U[1, 10].
    Summed in FP64 and stored as FP32, row-major [y][x].
    """
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0, width, n_bumps)
    cy = rng.uniform(0, height, n_bumps)
    s = rng.uniform(3.0, 12.0, n_bumps)
    h = rng.uniform(1.0, 10.0, n_bumps)
    gy, gx = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64), indexing="ij")
    acc = np.zeros((height, width), dtype=np.float64)
    for b in range(n_bumps):
        acc += h[b] * np.exp(-((gx - cx[b]) ** 2 + (gy - cy[b]) ** 2) / (2.0 * s[b] ** 2))
    return acc.astype(np.float32)


def obstacle_field(n: int = 32, seed: int = SEED_OBSTACLES, start=(0.0, 0.0, 1.5), goal=(8.0, 0.0, 1.5),
                   clearance: float = 0.5) -> np.ndarray:
    """n spheres (cx, cy, cz, r): centres ~ U([1,7] x [-3,3] x [0,3]), radii ~ U[0.3, 1.0],
    rejected when the start or goal lies within r + clearance."""
    rng = np.random.default_rng(seed)
    out = []
    start = np.asarray(start)
    goal = np.asarray(goal)
    while len(out) < n:
        c = rng.uniform([1.0, -3.0, 0.0], [7.0, 3.0, 3.0])
        r = rng.uniform(0.3, 1.0)
        if np.linalg.norm(c - start) < r + clearance or np.linalg.norm(c - goal) < r + clearance:
            continue
        out.append([c[0], c[1], c[2], r])
    return np.asarray(out, dtype=np.float64)


# ------------------------------------------------------------------------ workloads

def linear_double_integrator(K: int = 4096, T: int = 20, nu: float = 2.0, lam: float = 1.0,
                             sigma: float = 1.0, R: Optional[float] = None) -> Workload:
    """Test system: x = (position, velocity), one acceleration input, dt = 0.1.

    q(x) = x^T Q x with Q = I, phi(x) = x^T Qf x with Qf = 10 I.  R defaults to the
    coupled value lam / sigma (noise-cost coupling, Section II)."""
    if R is None:
        R = lam / sigma
    params = dict(A=np.array([[0.0, 1.0], [0.0, 0.0]]), B=np.array([[0.0], [1.0]]),
                  Q=np.eye(2), Qf=10.0 * np.eye(2))
    return Workload(name="linear", system=SYS_LINEAR, n=2, m=1, K=K, T=T, dt=0.1,
                    sigma=np.array([[sigma]]), nu=nu, lam=lam, R=np.array([[R]]),
                    u_init=np.zeros(1), params=params, x0=np.array([1.0, 0.0]))


def cartpole(nu: float = 1.0, K: int = 1000, T: int = 100, x0_index: int = 0) -> Workload:
    """Cart-pole: state (x, xdot, theta, thetadot), theta = 0 upright, one force input.

    Cart mass 1.0, pole mass 0.1, pole half-length 0.5, g = 9.81, dt = 0.02, Sigma = 1,
    lambda = 1, q = x^T diag(1, 0.1, 10, 0.1) x, R = 0.01; x0 ~ U[-0.5, 0.5]^4."""
    params = dict(mass_cart=1.0, mass_pole=0.1, half_length=0.5, gravity=9.81,
                  q_diag=np.array([1.0, 0.1, 10.0, 0.1]), qf_diag=np.zeros(4))
    x0 = uniform_states(max(x0_index + 1, 5), [-0.5] * 4, [0.5] * 4)[x0_index]
    return Workload(name="cartpole", system=SYS_CARTPOLE, n=4, m=1, K=K, T=T, dt=0.02,
                    sigma=np.array([[1.0]]), nu=nu, lam=1.0, R=np.array([[0.01]]),
                    u_init=np.zeros(1), params=params, x0=x0, control_steps=200)


SWINGUP_DT = 0.02          # the controller's 50 Hz re-optimisation period (Section V)
SWINGUP_NOISE = 0.01       # 1/sqrt(rho) of the swing-up experiment (Section V-A)
SWINGUP_HALF_LENGTH = 1.0  # pole half-length (builder-choice: the paper gives no pole model)


def cartpole_swingup(nu: float = 1.0, K: int = 1000, T: int = 50, control_steps: int = 500) -> Workload:
    """The cart-pole swing-up of Section V-A: velocity-command cart (pddot = 10 (u - pdot)),
    q = p^2 + 500 (1 + cos theta)^2 + thetadot^2 + pdot^2, R = 1, 1/sqrt(rho) = 0.01,
    1 s horizon (T = 50 at dt = 0.02), 10 s run (500 control steps), pole hanging at rest.

    The disturbance parameter 1/sqrt(rho) is read as the standard deviation of the per-step
    control perturbation, Sigma = 1e-4, and lambda follows the noise-cost coupling
    Sigma = lambda R^-1 in the per-step cost units used here, lambda = 1e-4.  Pole: a uniform
    rod of half-length 1 m, g = 9.81 (builder-choice).  Under these readings the natural
    variance (nu = 1) never brings the pole up in the 10 s, as Section V-A reports; the
    alternative readings and their outcomes are tabulated with the design notes."""
    sigma = SWINGUP_NOISE ** 2
    params = dict(gain=10.0, half_length=SWINGUP_HALF_LENGTH, gravity=9.81, w_pos=1.0, w_angle=500.0, w_vel=1.0,
                  w_rate=1.0)
    return Workload(name="cartpole_swingup", system=SYS_CARTPOLE_SWINGUP, n=4, m=1, K=K, T=T, dt=SWINGUP_DT,
                    sigma=np.array([[sigma]]), nu=nu, lam=sigma * 1.0, R=np.array([[1.0]]),
                    u_init=np.zeros(1), params=params, x0=np.zeros(4), control_steps=control_steps)


# Temperatures not given for these systems: calibrated so that the effective sample size is
# 5 % of K at iteration 0 from the initial state (tests/golden/calibrate_lambda.py).
BICYCLE_LAMBDA = 130.0


def bicycle(K: int = 4096, T: int = 100, nu: float = 2.0, lam: float = BICYCLE_LAMBDA,
            x0_index: int = 0, the_map: Optional[np.ndarray] = None) -> Workload:
    """Kinematic bicycle: state (x, y, yaw, v, steer), controls (accel, steer rate).

    Wheelbase 2.5 m, dt = 0.05, Sigma = diag(0.5, 0.3), nu = 2, R = 0.01 I.
    q = bilinear(map, x, y) + (v - 5)^2 on a 256x256 map of 0.5 m cells.
    The steering angle entering tan() is clamped to +-0.6 rad (builder-choice)."""
    if the_map is None:
        the_map = cost_map()
    rng = np.random.default_rng(SEED_X0 + 1)
    yaws = rng.uniform(-math.pi, math.pi, max(x0_index + 1, 5))
    params = dict(wheelbase=2.5, v_target=5.0, w_speed=1.0, cell_size=0.5, steer_limit=0.6, map=the_map)
    x0 = np.array([64.0, 64.0, yaws[x0_index], 0.0, 0.0])
    return Workload(name="bicycle", system=SYS_BICYCLE, n=5, m=2, K=K, T=T, dt=0.05,
                    sigma=np.diag([0.5, 0.3]), nu=nu, lam=lam, R=0.01 * np.eye(2),
                    u_init=np.zeros(2), params=params, x0=x0)


QUAD_MASS = 1.0
QUAD_GRAVITY = 9.81
QUAD_HOVER = QUAD_MASS * QUAD_GRAVITY / 4.0
QUADROTOR_LAMBDA = {1.0: 410.0, 2.0: 420.0, 4.0: 460.0}


QUAD_CRASH_COST = 1000.0    # the crash indicator's weight in the quadrotor cost (Section V-C)


def quadrotor_params(obstacles: Optional[np.ndarray] = None, crash_cost: float = 0.0) -> Dict:
    """'+' rotor layout, arm 0.2 m, yaw-torque coefficient 0.01 m, inertia diag(0.01, 0.01, 0.02).

    q = w_goal * |p - goal|^2 + w_obs * sum_j max(0, (r_j + margin)^2 - |p - c_j|^2)^2,
    plus crash_cost * C (crash indicator, ground at z = 0) when crash_cost > 0."""
    if obstacles is None:
        obstacles = obstacle_field()
    return dict(mass=QUAD_MASS, gravity=QUAD_GRAVITY, arm=0.2, yaw_coef=0.01,
                inertia=np.array([0.01, 0.01, 0.02]), goal=np.array([8.0, 0.0, 1.5]),
                w_goal=1.0, w_obs=1000.0, obs_margin=0.1, obstacles=obstacles,
                crash_cost=crash_cost, ground_z=0.0)


def quadrotor(nu: float = 2.0, K: int = 16384, T: int = 150, lam: Optional[float] = None,
              obstacles: Optional[np.ndarray] = None, crash: bool = False) -> Workload:
    """Quadrotor rigid body: state (p, v, roll/pitch/yaw, body rates), four rotor thrusts.

    Mass 1.0, inertia diag(0.01, 0.01, 0.02), dt = 0.01, R = 0.1 I, Sigma = 0.25 I N^2
    (builder-choice), u_init = hover thrust; start (0, 0, 1.5), goal (8, 0, 1.5)."""
    if lam is None:
        lam = QUADROTOR_LAMBDA.get(float(nu), 420.0)
    x0 = np.zeros(12)
    x0[2] = 1.5
    return Workload(name="quadrotor", system=SYS_QUADROTOR, n=12, m=4, K=K, T=T, dt=0.01,
                    sigma=0.25 * np.eye(4), nu=nu, lam=lam, R=0.1 * np.eye(4),
                    u_init=np.full(4, QUAD_HOVER),
                    params=quadrotor_params(obstacles, QUAD_CRASH_COST if crash else 0.0), x0=x0)


def quadrotor_mlp(net, nu: float = 2.0, K: int = 16384, T: int = 100, lam: Optional[float] = None) -> Workload:
    """Learned-dynamics quadrotor: the quadrotor workload with x <- x + MLP(x, u); ``net`` is
    the network object the consumer uses (a GPU handle or an oracle network)."""
    wl = quadrotor(nu=nu, K=K, T=T, lam=lam)
    return wl.replace(name="quadrotor_mlp", system=SYS_QUADROTOR_MLP, params=dict(wl.params, mlp=net))


# ------------------------------------------------------------------ MLP training data

MLP_BOX_LO = np.array([-5, -5, -5, -2, -2, -2, -0.5, -0.5, -0.5, -2, -2, -2], dtype=np.float64)
MLP_BOX_HI = -MLP_BOX_LO


def mlp_training_inputs(n: int = 1_000_000, seed: int = SEED_MLP_DATA, control_std: float = 1.0):
    """(state, control) pairs for the learned-dynamics surrogate: states uniform in the
    operating box, controls Gaussian around hover thrust.  Targets are produced by each
    side's own quadrotor dynamics, not here."""
    rng = np.random.default_rng(seed)
    x = MLP_BOX_LO + (MLP_BOX_HI - MLP_BOX_LO) * rng.random((n, 12))
    u = QUAD_HOVER + control_std * rng.standard_normal((n, 4))
    return x, u


def mlp_init_weights(seed: int = SEED_MLP_INIT, hidden: int = 128, n_in: int = 16, n_out: int = 12):
    """Initial MLP weights (Glorot & Bengio 2010 uniform, zero biases): W1 (h, n_in),
    W2 (h, h), W3 (n_out, h); FP32 values, returned as float64 arrays."""
    rng = np.random.default_rng(seed)

    def glorot(fan_out, fan_in):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, (fan_out, fan_in)).astype(np.float32).astype(np.float64)

    W1 = glorot(hidden, n_in)
    W2 = glorot(hidden, hidden)
    W3 = glorot(n_out, hidden)
    return dict(W1=W1, b1=np.zeros(hidden), W2=W2, b2=np.zeros(hidden), W3=W3, b3=np.zeros(n_out))


def minibatch_order(n: int, epochs: int, seed: int = SEED_MLP_DATA + 1):
    """Sample order of each training epoch (a seeded permutation per epoch)."""
    rng = np.random.default_rng(seed)
    return [rng.permutation(n) for _ in range(epochs)]


# --------------------------------------------------------------------- serving trace

def serving_mix(n_controllers: int = 256, seed: int = SEED_SERVING):
    """Controller mix: system ~ U{cartpole, bicycle, quadrotor}, K ~ U{512, 2048, 8192, 16384},
    T ~ U{50, 100, 200}."""
    rng = np.random.default_rng(seed)
    systems = rng.integers(0, 3, n_controllers)
    Ks = rng.choice([512, 2048, 8192, 16384], n_controllers)
    Ts = rng.choice([50, 100, 200], n_controllers)
    return [(int(s), int(k), int(t)) for s, k, t in zip(systems, Ks, Ts)]


def poisson_arrivals(n_controllers: int, rate_hz: float, duration_s: float, seed: int = SEED_SERVING + 1):
    """Sorted (time, controller) arrivals: an independent Poisson process per controller."""
    rng = np.random.default_rng(seed)
    events = []
    for c in range(n_controllers):
        t = rng.exponential(1.0 / rate_hz)
        while t < duration_s:
            events.append((t, c))
            t += rng.exponential(1.0 / rate_hz)
    events.sort()
    return events


def serving_sessions(n_controllers: int = 256, start_s: float = 3.0, min_life_s: float = 4.0, max_life_s: float = 8.0,
                     seed: int = SEED_SERVING + 2):
    """Controller sessions: controller c arrives at t_start ~ U[0, start_s) and stays for
    U[min_life_s, max_life_s) seconds.  Returns (t_start, t_end) arrays."""
    rng = np.random.default_rng(seed)
    t0 = rng.uniform(0.0, start_s, n_controllers)
    return t0, t0 + rng.uniform(min_life_s, max_life_s, n_controllers)


def session_arrivals(t_start, t_end, rate_hz: float, seed: int = SEED_SERVING + 3):
    """Sorted (time, session) arrivals: an independent Poisson process per session over its
    lifetime [t_start, t_end)."""
    rng = np.random.default_rng(seed)
    events = []
    for c, (a, b) in enumerate(zip(t_start, t_end)):
        t = a + rng.exponential(1.0 / rate_hz)
        while t < b:
            events.append((t, c))
            t += rng.exponential(1.0 / rate_hz)
    events.sort()
    return events
