"""Dynamics and state costs of the test systems, FP64, vectorised over samples
(test infrastructure only).

The paper's problem statement (Section II, the control-affine dynamics, its
partition and the cost functional) only fixes the *form*: x' = f(x) + G(x) u,
a state cost q(x) and a terminal cost phi(x).  Algorithm 1 steps the dynamics with
one explicit Euler step per time step, x_{i+1} = x_i + (f + G v_i) dt, which is
``euler_step`` below.  The concrete systems are synthetic stand-ins for the
paper's experiments (Section V); their constants are builder choices frozen in
``workloads``.
"""
import numpy as np


def euler_step(system, x, v, dt):
    """Algorithm 1's transition: x + (f(x) + G(x) v) dt.  A system with its own discrete
    ``step`` (the learned one-step model) uses that instead."""
    if hasattr(system, "step"):
        return system.step(x, v, dt)
    return x + dt * system.xdot(x, v)


class Linear:
    """x' = A x + B v; q = x^T Q x; phi = x^T Qf x."""

    def __init__(self, params):
        self.A = np.asarray(params["A"], float)
        self.B = np.asarray(params["B"], float)
        self.Q = np.asarray(params["Q"], float)
        self.Qf = np.asarray(params["Qf"], float)

    def xdot(self, x, v):
        return x @ self.A.T + v @ self.B.T

    def q(self, x):
        return np.einsum("ki,ij,kj->k", x, self.Q, x)

    def phi(self, x):
        return np.einsum("ki,ij,kj->k", x, self.Qf, x)


class CartPole:
    """Frictionless cart with a uniform pole (half-length l, inertia about the pivot
    (4/3) m_p l^2), theta = 0 upright, force input.  State (x, xdot, theta, thetadot).

    Lagrangian equations of motion with M = m_c + m_p:
      h          = (F + m_p l thetadot^2 sin theta) / M
      thetaddot  = (g sin theta - cos theta h) / (l (4/3 - m_p cos^2 theta / M))
      xddot      = h - m_p l thetaddot cos theta / M
    q = x^T diag(q_diag) x, phi = x^T diag(qf_diag) x.
    """

    def __init__(self, params):
        self.mc = params["mass_cart"]
        self.mp = params["mass_pole"]
        self.l = params["half_length"]
        self.g = params["gravity"]
        self.qd = np.asarray(params["q_diag"], float)
        self.qfd = np.asarray(params["qf_diag"], float)

    def xdot(self, x, v):
        F = v[:, 0]
        xd, th, thd = x[:, 1], x[:, 2], x[:, 3]
        M = self.mc + self.mp
        s, c = np.sin(th), np.cos(th)
        h = (F + self.mp * self.l * thd * thd * s) / M
        thdd = (self.g * s - c * h) / (self.l * (4.0 / 3.0 - self.mp * c * c / M))
        xdd = h - self.mp * self.l * thdd * c / M
        return np.stack([xd, xdd, thd, thdd], axis=1)

    def q(self, x):
        return (x * x) @ self.qd

    def phi(self, x):
        return (x * x) @ self.qfd

    # invariants used by the tests (not by the method)
    def energy(self, x):
        M = self.mc + self.mp
        xd, th, thd = x[..., 1], x[..., 2], x[..., 3]
        return (0.5 * M * xd ** 2 + self.mp * self.l * xd * thd * np.cos(th)
                + (2.0 / 3.0) * self.mp * self.l ** 2 * thd ** 2 + self.mp * self.g * self.l * np.cos(th))

    def momentum(self, x):
        M = self.mc + self.mp
        return M * x[..., 1] + self.mp * self.l * x[..., 3] * np.cos(x[..., 2])


def bilinear(the_map, gx, gy):
    """Bilinear interpolation of a row-major [y][x] grid at fractional cell coordinates,
    clamped to the grid.  Exact at cell centres; exact for affine fields."""
    H, W = the_map.shape
    gx = np.clip(gx, 0.0, W - 1.0)
    gy = np.clip(gy, 0.0, H - 1.0)
    i0 = np.minimum(np.floor(gx), W - 2).astype(np.int64)
    j0 = np.minimum(np.floor(gy), H - 2).astype(np.int64)
    fx = gx - i0
    fy = gy - j0
    m = np.asarray(the_map, dtype=np.float64)
    top = (1.0 - fx) * m[j0, i0] + fx * m[j0, i0 + 1]
    bot = (1.0 - fx) * m[j0 + 1, i0] + fx * m[j0 + 1, i0 + 1]
    return (1.0 - fy) * top + fy * bot


class Bicycle:
    """Kinematic bicycle, state (x, y, yaw, v, delta), controls (a, omega):
    x' = v cos yaw, y' = v sin yaw, yaw' = v tan(clamp(delta)) / L, v' = a, delta' = omega.
    q = map(x / cell, y / cell) + w_speed (v - v_target)^2; phi = 0."""

    def __init__(self, params):
        self.L = params["wheelbase"]
        self.vt = params["v_target"]
        self.ws = params["w_speed"]
        self.cell = params["cell_size"]
        self.lim = params["steer_limit"]
        self.map = np.asarray(params["map"])

    def xdot(self, x, v):
        yaw, vel, dl = x[:, 2], x[:, 3], x[:, 4]
        if self.lim > 0:
            dl = np.clip(dl, -self.lim, self.lim)
        return np.stack([vel * np.cos(yaw), vel * np.sin(yaw), vel * np.tan(dl) / self.L,
                         v[:, 0], v[:, 1]], axis=1)

    def q(self, x):
        return bilinear(self.map, x[:, 0] / self.cell, x[:, 1] / self.cell) + self.ws * (x[:, 3] - self.vt) ** 2

    def phi(self, x):
        return np.zeros(x.shape[0])


def rot_zyx(roll, pitch, yaw):
    """Body-to-world rotation R = Rz(yaw) Ry(pitch) Rx(roll), shape (..., 3, 3)."""
    cr, sr = np.cos(roll), np.sin(roll)
    cp, sp = np.cos(pitch), np.sin(pitch)
    cy, sy = np.cos(yaw), np.sin(yaw)
    R = np.empty(np.shape(roll) + (3, 3))
    R[..., 0, 0] = cy * cp
    R[..., 0, 1] = cy * sp * sr - sy * cr
    R[..., 0, 2] = cy * sp * cr + sy * sr
    R[..., 1, 0] = sy * cp
    R[..., 1, 1] = sy * sp * sr + cy * cr
    R[..., 1, 2] = sy * sp * cr - cy * sr
    R[..., 2, 0] = -sp
    R[..., 2, 1] = cp * sr
    R[..., 2, 2] = cp * cr
    return R


class Quadrotor:
    """Rigid-body quadrotor, state (p[3], v[3], roll, pitch, yaw, body rates w[3]),
    controls = four rotor thrusts in a '+' layout (rotor 1 on +x, 2 on +y, 3 on -x, 4 on -y).

      p' = v
      v' = (sum f / m) R(eta) e3 - g e3
      eta' = W(eta)^-1 w            (ZYX Euler-angle rates)
      w' = J^-1 (tau - w x J w),    tau = (l (f2 - f4), l (f3 - f1), kappa (f1 - f2 + f3 - f4))
    q = w_goal |p - goal|^2 + w_obs sum_j max(0, (r_j + margin)^2 - |p - c_j|^2)^2, phi = 0.
    With crash_cost > 0 a rollout that crashes stops moving and pays crash_cost at every
    remaining step (``crashed``, applied by the rollout in oracle.mppi).
    """

    def __init__(self, params):
        self.m = params["mass"]
        self.g = params["gravity"]
        self.arm = params["arm"]
        self.kap = params["yaw_coef"]
        self.J = np.asarray(params["inertia"], float)
        self.goal = np.asarray(params["goal"], float)
        self.wg = params["w_goal"]
        self.wo = params["w_obs"]
        self.margin = params["obs_margin"]
        self.obs = np.asarray(params["obstacles"], float).reshape(-1, 4)
        # crash indicator C of Section V-C (0 disables it): cost per step once crashed
        self.crash_cost = float(params.get("crash_cost", 0.0))
        self.ground_z = float(params.get("ground_z", 0.0))

    def crashed(self, x):
        """C = 1: below the ground plane or inside an obstacle (its radius, no margin)."""
        p = x[:, 0:3]
        hit = p[:, 2] < self.ground_z
        for cx, cy, cz, r in self.obs:
            hit = hit | ((p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2 + (p[:, 2] - cz) ** 2 < r * r)
        return hit

    def xdot(self, x, f):
        vel = x[:, 3:6]
        roll, pitch, yaw = x[:, 6], x[:, 7], x[:, 8]
        w = x[:, 9:12]
        R = rot_zyx(roll, pitch, yaw)
        thrust = f.sum(axis=1)
        acc = (thrust / self.m)[:, None] * R[:, :, 2]
        acc[:, 2] -= self.g
        sr, cr = np.sin(roll), np.cos(roll)
        tp, cp = np.tan(pitch), np.cos(pitch)
        eta_dot = np.stack([w[:, 0] + sr * tp * w[:, 1] + cr * tp * w[:, 2],
                            cr * w[:, 1] - sr * w[:, 2],
                            (sr * w[:, 1] + cr * w[:, 2]) / cp], axis=1)
        tau = np.stack([self.arm * (f[:, 1] - f[:, 3]),
                        self.arm * (f[:, 2] - f[:, 0]),
                        self.kap * (f[:, 0] - f[:, 1] + f[:, 2] - f[:, 3])], axis=1)
        Jw = w * self.J
        w_dot = (tau - np.cross(w, Jw)) / self.J
        return np.concatenate([vel, acc, eta_dot, w_dot], axis=1)

    def q(self, x):
        p = x[:, 0:3]
        d = p - self.goal
        cost = self.wg * np.einsum("ki,ki->k", d, d)
        for cx, cy, cz, r in self.obs:
            dd = (p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2 + (p[:, 2] - cz) ** 2
            pen = np.maximum(0.0, (r + self.margin) ** 2 - dd)
            cost = cost + self.wo * pen * pen
        return cost

    def phi(self, x):
        return np.zeros(x.shape[0])


class CartPoleSwingUp:
    """The cart-pole of the swing-up experiment (Section V-A): the control is a desired cart
    velocity, tracked as pddot = gain (u - pdot); the pole is a uniform rod of half-length l
    on a pivot that the cart accelerates, theta = 0 hanging down and theta = pi upright:
      thetaddot = -(3 / (4 l)) (g sin theta + pddot cos theta)
    (rotation about the pivot, inertia (4/3) m l^2, under gravity and the pivot's
    acceleration).  State (p, pdot, theta, thetadot).
    q = w_pos p^2 + w_angle (1 + cos theta)^2 + w_rate thetadot^2 + w_vel pdot^2, phi = 0."""

    def __init__(self, params):
        self.gain = params["gain"]
        self.l = params["half_length"]
        self.g = params["gravity"]
        self.w_pos, self.w_angle = params["w_pos"], params["w_angle"]
        self.w_vel, self.w_rate = params["w_vel"], params["w_rate"]

    def xdot(self, x, v):
        pd, th, thd = x[:, 1], x[:, 2], x[:, 3]
        pdd = self.gain * (v[:, 0] - pd)
        thdd = -(3.0 / (4.0 * self.l)) * (self.g * np.sin(th) + pdd * np.cos(th))
        return np.stack([pd, pdd, thd, thdd], axis=1)

    def q(self, x):
        p, pd, th, thd = x[:, 0], x[:, 1], x[:, 2], x[:, 3]
        return (self.w_pos * p * p + self.w_angle * (1.0 + np.cos(th)) ** 2
                + self.w_rate * thd * thd + self.w_vel * pd * pd)

    def phi(self, x):
        return np.zeros(x.shape[0])

    # invariant used by the tests (not by the method): pole energy per unit mass in the
    # cart's frame, (2/3) l^2 thetadot^2 - g l cos theta
    def pole_energy(self, x):
        return (2.0 / 3.0) * self.l ** 2 * x[..., 3] ** 2 - self.g * self.l * np.cos(x[..., 2])


def make(workload):
    from workloads import SYS_LINEAR, SYS_CARTPOLE, SYS_BICYCLE, SYS_QUADROTOR, SYS_CARTPOLE_SWINGUP
    table = {SYS_LINEAR: Linear, SYS_CARTPOLE: CartPole, SYS_BICYCLE: Bicycle, SYS_QUADROTOR: Quadrotor,
             SYS_CARTPOLE_SWINGUP: CartPoleSwingUp}
    if workload.system not in table:
        raise ValueError(f"oracle has no analytic system {workload.system}")
    return table[workload.system](workload.params)
