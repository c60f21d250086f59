"""Pins of the oracle's dynamics and costs (CPU only), by physics and geometry rather
than by retyping the equations:

* cart-pole: horizontal momentum and energy are conserved with zero force, momentum
  grows by F t and energy by F (x(t) - x(0)) under a constant force F;
* quadrotor: hover is an equilibrium; a torque-free rotation conserves the world-frame
  angular momentum R J w and the kinetic energy; the Euler-angle rates reproduce
  dR/dt = R [w]x; torques equal sum_i r_i x (f_i e3) for the '+' rotor layout;
* bicycle: constant steer traces a circle of radius L / tan(delta);
* bilinear map: exact at cell centres and for affine fields, clamped outside.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W
from oracle import systems


def _flow(sys_, x0, u, t_end):
    f = lambda t, x: sys_.xdot(x[None, :], np.asarray(u, float)[None, :])[0]
    return solve_ivp(f, (0, t_end), x0, rtol=1e-11, atol=1e-12, dense_output=True)


def test_cartpole_conservation_laws():
    cp = systems.CartPole(W.cartpole().params)
    rng = np.random.default_rng(0)
    for _ in range(4):
        x0 = rng.uniform(-1.5, 1.5, 4)
        sol = _flow(cp, x0, [0.0], 2.0)
        xs = sol.y.T
        assert np.allclose(cp.momentum(xs), cp.momentum(x0), atol=1e-8)
        assert np.allclose(cp.energy(xs), cp.energy(x0), atol=1e-8)
        F = 0.7
        sol = _flow(cp, x0, [F], 1.0)
        xe = sol.y[:, -1]
        assert cp.momentum(xe) == pytest.approx(cp.momentum(x0) + F * 1.0, abs=1e-8)
        assert cp.energy(xe) == pytest.approx(cp.energy(x0) + F * (xe[0] - x0[0]), abs=1e-8)


def test_cartpole_upright_equilibrium_and_fall_direction():
    cp = systems.CartPole(W.cartpole().params)
    assert np.allclose(cp.xdot(np.zeros((1, 4)), np.zeros((1, 1))), 0)
    xd = cp.xdot(np.array([[0, 0, 0.1, 0]]), np.zeros((1, 1)))[0]
    assert xd[3] > 0          # tilted pole accelerates away from upright


def _quad(**over):
    p = W.quadrotor_params()
    p = dict(p, **over)
    return systems.Quadrotor(p)


def test_quadrotor_hover_is_an_equilibrium():
    q = _quad()
    x = np.zeros((1, 12))
    x[0, :3] = [1.0, -2.0, 3.0]
    assert np.allclose(q.xdot(x, np.full((1, 4), W.QUAD_HOVER)), 0, atol=1e-15)


def test_quadrotor_torque_free_rotation_invariants():
    q = _quad(gravity=0.0)
    rng = np.random.default_rng(1)
    x0 = np.zeros(12)
    x0[6:9] = rng.uniform(-0.4, 0.4, 3)
    x0[9:12] = rng.uniform(-2, 2, 3)
    sol = _flow(q, x0, np.zeros(4), 0.6)
    J = q.J
    for t in np.linspace(0, 0.6, 7):
        x = sol.sol(t)
        R = systems.rot_zyx(*x[6:9])
        assert np.allclose(R @ (J * x[9:12]), systems.rot_zyx(*x0[6:9]) @ (J * x0[9:12]), atol=1e-8)
        assert 0.5 * np.sum(J * x[9:12] ** 2) == pytest.approx(0.5 * np.sum(J * x0[9:12] ** 2), rel=1e-9)


def test_quadrotor_euler_rates_match_rotation_kinematics():
    q = _quad()
    rng = np.random.default_rng(2)
    for _ in range(5):
        x = np.zeros(12)
        x[6:9] = rng.uniform(-0.6, 0.6, 3)
        x[9:12] = rng.uniform(-1, 1, 3)
        eta_dot = q.xdot(x[None], np.zeros((1, 4)))[0, 6:9]
        h = 1e-6
        dR = (systems.rot_zyx(*(x[6:9] + h * eta_dot)) - systems.rot_zyx(*(x[6:9] - h * eta_dot))) / (2 * h)
        w = x[9:12]
        skew = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        assert np.allclose(dR, systems.rot_zyx(*x[6:9]) @ skew, atol=1e-8)


def test_quadrotor_thrust_and_torques():
    q = _quad()
    rng = np.random.default_rng(3)
    f = rng.uniform(1, 4, 4)
    x = np.zeros(12)
    x[6:9] = rng.uniform(-0.5, 0.5, 3)
    xd = q.xdot(x[None], f[None])[0]
    R = systems.rot_zyx(*x[6:9])
    assert np.allclose(xd[3:6], f.sum() / q.m * R[:, 2] - np.array([0, 0, q.g]), atol=1e-14)
    arm = q.arm
    pos = np.array([[arm, 0, 0], [0, arm, 0], [-arm, 0, 0], [0, -arm, 0]])
    tau = sum(np.cross(pos[i], [0, 0, f[i]]) for i in range(4))
    tau[2] = q.kap * (f[0] - f[1] + f[2] - f[3])
    assert np.allclose(xd[9:12], tau / q.J, atol=1e-12)     # at w = 0 the gyroscopic term vanishes


def test_bicycle_circle_and_line():
    p = W.bicycle().params
    b = systems.Bicycle(p)
    delta, v, L = 0.3, 4.0, p["wheelbase"]
    x0 = np.array([10.0, 20.0, 0.4, v, delta])
    sol = _flow(b, x0, [0.0, 0.0], 3.0)
    rad = L / np.tan(delta)
    cx, cy = x0[0] - rad * np.sin(x0[2]), x0[1] + rad * np.cos(x0[2])
    xs = sol.y.T
    assert np.allclose(np.hypot(xs[:, 0] - cx, xs[:, 1] - cy), rad, atol=1e-8)
    assert xs[-1, 2] == pytest.approx(x0[2] + v * np.tan(delta) / L * 3.0, abs=1e-8)
    # straight line: one Euler step is exact
    x = np.array([[1.0, 2.0, 0.7, 3.0, 0.0]])
    assert np.allclose(systems.euler_step(b, x, np.zeros((1, 2)), 0.5)[0, :2],
                       [1.0 + 1.5 * np.cos(0.7), 2.0 + 1.5 * np.sin(0.7)], atol=1e-15)
    # steering beyond the limit saturates
    xd1 = b.xdot(np.array([[0, 0, 0, 2.0, 1.2]]), np.zeros((1, 2)))
    xd2 = b.xdot(np.array([[0, 0, 0, 2.0, p["steer_limit"]]]), np.zeros((1, 2)))
    assert np.allclose(xd1, np.where(np.arange(5) == 4, 0, xd2))


def test_bilinear_map():
    rng = np.random.default_rng(4)
    m = rng.uniform(0, 10, (6, 9))
    j, i = np.meshgrid(np.arange(6), np.arange(9), indexing="ij")
    assert np.allclose(systems.bilinear(m, i.ravel().astype(float), j.ravel().astype(float)), m.ravel(), atol=1e-14)
    aff = 2.0 + 0.5 * i - 1.25 * j
    gx, gy = rng.uniform(0, 8, 100), rng.uniform(0, 5, 100)
    assert np.allclose(systems.bilinear(aff, gx, gy), 2.0 + 0.5 * gx - 1.25 * gy, atol=1e-12)
    assert systems.bilinear(m, np.array([-3.0]), np.array([100.0]))[0] == m[5, 0]


def test_bicycle_cost_uses_cells_of_the_map():
    wl = W.bicycle()
    b = systems.Bicycle(wl.params)
    x = np.array([[3.0, 5.5, 0, 5.0, 0]])    # cell (6, 11), on target speed
    assert b.q(x)[0] == pytest.approx(float(wl.params["map"][11, 6]), rel=1e-7)


def test_quadrotor_barrier():
    q = _quad()
    ob = q.obs[0]
    x = np.zeros((1, 12))
    x[0, :3] = q.goal
    assert q.q(x)[0] == pytest.approx(sum(q.wo * max(0.0, (o[3] + q.margin) ** 2 - np.sum((q.goal - o[:3]) ** 2)) ** 2
                                          for o in q.obs), abs=1e-9)
    x[0, :3] = ob[:3]
    assert q.q(x)[0] >= q.wo * ((ob[3] + q.margin) ** 2) ** 2


# ------------------------------------------------------------- cart-pole swing-up
def _swingup():
    return systems.CartPoleSwingUp(W.cartpole_swingup().params)


def test_swingup_cart_tracks_the_commanded_velocity():
    """pddot = 10 (u - pdot): pdot(t) = u + (pdot0 - u) exp(-10 t), whatever the pole does."""
    su = _swingup()
    x0 = np.array([0.3, -0.5, 2.0, 1.0])
    sol = _flow(su, x0, [1.5], 1.0)
    t = np.linspace(0, 1, 11)
    assert np.allclose(sol.sol(t)[1], 1.5 + (-0.5 - 1.5) * np.exp(-10.0 * t), atol=1e-8)


def test_swingup_pendulum_period_and_energy_at_constant_cart_velocity():
    """With pdot = u the pivot moves uniformly, so the pole is a free physical pendulum:
    its energy per unit mass (2/3) l^2 thetadot^2 - g l cos theta is conserved, and small
    swings have period 2 pi sqrt(I / (m g l)) = 2 pi sqrt(4 l / (3 g)) for a uniform rod."""
    su = _swingup()
    l, g = W.SWINGUP_HALF_LENGTH, 9.81
    E = lambda x: (2.0 / 3.0) * l * l * x[3] ** 2 - g * l * np.cos(x[2])
    rng = np.random.default_rng(4)
    for _ in range(3):
        x0 = np.array([0.0, 0.7, rng.uniform(-3, 3), rng.uniform(-4, 4)])
        sol = _flow(su, x0, [0.7], 2.0)
        xe = sol.y[:, -1]
        assert abs(E(xe) - E(x0)) < 1e-8
        assert abs(xe[0] - 0.7 * 2.0) < 1e-8
    sol = _flow(su, np.array([0.0, 0.0, 0.01, 0.0]), [0.0], 3.0)
    t = np.linspace(0, 3, 300001)
    th = sol.sol(t)[2]
    up = t[1:][(th[:-1] < 0) & (th[1:] >= 0)]           # upward zero crossings
    assert np.allclose(np.diff(up), 2 * np.pi * np.sqrt(4 * l / (3 * g)), rtol=1e-4)


def test_swingup_pivot_acceleration_drives_the_pole():
    """Power balance in the cart's frame: the pseudo-force -m pddot on the centre of mass
    (lever l cos theta) changes the pole's energy at the rate -l pddot thetadot cos theta;
    and a hanging pole swings backwards (theta < 0) when the cart accelerates forwards."""
    su = _swingup()
    l, g = W.SWINGUP_HALF_LENGTH, 9.81

    def f(t, z):
        x = z[:4]
        xd = su.xdot(x[None, :], np.array([[2.0 * np.sin(3 * t)]]))[0]
        return np.concatenate([xd, [-l * xd[1] * x[3] * np.cos(x[2])]])

    rng = np.random.default_rng(5)
    for _ in range(3):
        x0 = rng.uniform(-2, 2, 4)
        sol = solve_ivp(f, (0, 2), np.concatenate([x0, [0.0]]), rtol=1e-11, atol=1e-12)
        xe, work = sol.y[:4, -1], sol.y[4, -1]
        E = lambda x: (2.0 / 3.0) * l * l * x[3] ** 2 - g * l * np.cos(x[2])
        assert abs(E(xe) - E(x0) - work) < 1e-7
    sol = _flow(su, np.zeros(4), [1.0], 0.1)
    assert sol.y[2, -1] < 0 and sol.y[1, -1] > 0


def test_swingup_cost_hanging_and_upright():
    """The pole hanging at rest costs 500 (1 + 1)^2 = 2000 per step (the running cost the
    paper reports when the pole is never swung up); upright at rest costs 0."""
    su = _swingup()
    assert su.q(np.zeros((1, 4)))[0] == 2000.0
    assert su.q(np.array([[0.0, 0.0, np.pi, 0.0]]))[0] < 1e-20
    assert np.array_equal(su.q(np.array([[2.0, 0.0, np.pi, 0.0]])), su.q(np.array([[-2.0, 0.0, np.pi, 0.0]])))
