"""Pins of the oracle's MPPI iteration (CPU only): invariants of the update law and
of Algorithm 1, closed forms in the linear-quadratic case, and the exact shard merge."""
import numpy as np
import pytest

import workloads as W
from oracle import lqr, mppi, noise, systems


def _se(r):
    """Monte-Carlo standard error of the self-normalised estimate, from the weights."""
    return np.sqrt(np.einsum("k,ktj->tj", r.w ** 2, (r.du - r.dU[None]) ** 2))


def test_weights_are_a_distribution_peaked_at_the_best_sample():
    wl = W.cartpole(nu=2.0, K=500, T=30)
    r = mppi.iteration(wl, wl.x0, mppi.initial_sequence(wl), 0)
    assert np.all(r.w >= 0) and abs(r.w.sum() - 1.0) < 1e-15 * wl.K
    assert np.argmax(r.w) == np.argmin(r.S) and r.eta >= 1.0
    assert r.rho == r.S.min()


def test_shifting_all_costs_changes_nothing():
    rng = np.random.default_rng(1)
    S = rng.uniform(0, 50, 200)
    du = rng.standard_normal((200, 5, 2))
    w1, _, _, d1, _ = mppi.weights_and_update(S, du, 3.0)
    w2, _, _, d2, _ = mppi.weights_and_update(S + 1e4, du, 3.0)
    assert np.allclose(w1, w2, rtol=1e-12) and np.allclose(d1, d2, rtol=1e-12)


def test_temperature_limits():
    rng = np.random.default_rng(2)
    S = rng.uniform(0, 50, 300)
    du = rng.standard_normal((300, 4, 1))
    _, _, _, hot, _ = mppi.weights_and_update(S, du, 1e12)
    assert np.allclose(hot, du.mean(axis=0), atol=1e-9)
    _, _, _, cold, _ = mppi.weights_and_update(S, du, 1e-9)
    assert np.array_equal(cold, du[np.argmin(S)])


def test_single_sample_takes_its_perturbation():
    wl = W.bicycle(K=1, T=20)
    U = mppi.initial_sequence(wl)
    r = mppi.iteration(wl, wl.x0, U, 4)
    assert np.array_equal(r.U, U + r.du[0])


def test_zero_noise_leaves_the_sequence_unchanged():
    wl = W.cartpole(K=64, T=25).replace(sigma=np.zeros((1, 1)))
    U = np.linspace(-1, 1, 25)[:, None]
    r = mppi.iteration(wl, wl.x0, U, 0)
    assert np.all(r.S == r.S[0]) and np.allclose(r.w, 1.0 / 64) and np.array_equal(r.U, U)


def test_nu_one_is_plain_mppi():
    wl = W.cartpole(nu=1.0, K=400, T=40)
    U = 0.3 * np.sin(np.arange(40))[:, None]
    r = mppi.iteration(wl, wl.x0, U, 9)
    U_plain, S_plain = mppi.plain_mppi_iteration(wl, wl.x0, U, 9)
    assert np.array_equal(r.S, S_plain)
    assert np.allclose(r.U, U_plain, rtol=0, atol=1e-15)


def test_common_random_numbers_across_nu():
    wl = W.quadrotor(nu=1.0, K=8, T=5)
    a = noise.control_noise(wl.seed, 3, 8, 5, wl.sigma, 1.0)
    b = noise.control_noise(wl.seed, 3, 8, 5, wl.sigma, 4.0)
    assert np.allclose(b, 2.0 * a, rtol=1e-15)


def test_non_finite_costs():
    du = np.ones((3, 2, 1))
    w, eta, rho, dU, st = mppi.weights_and_update(np.array([np.inf, 1.0, np.inf]), du, 1.0)
    assert st == mppi.STATUS_OK and np.array_equal(w, [0, 1, 0])
    w, eta, rho, dU, st = mppi.weights_and_update(np.array([np.inf] * 3), du, 1.0)
    assert st == mppi.STATUS_NUMERIC and not np.any(dU)


def test_shard_merge_is_exact():
    rng = np.random.default_rng(4)
    S = rng.uniform(0, 300, 1000)
    du = rng.standard_normal((1000, 6, 2))
    lam = 7.0
    _, _, _, full, _ = mppi.weights_and_update(S, du, lam)
    parts = []
    for sl in np.array_split(np.arange(1000), 7):
        rho_g = S[sl].min()
        e = np.exp(-(S[sl] - rho_g) / lam)
        parts.append((rho_g, e.sum(), np.einsum("k,ktj->tj", e, du[sl])))
    assert np.allclose(mppi.merge_shards(parts, lam), full, rtol=1e-13, atol=1e-15)


def test_control_step_emits_and_shifts():
    wl = W.bicycle(K=256, T=10).replace(n_iters=2)
    U = mppi.initial_sequence(wl) + 0.1
    u0, Us, it, res = mppi.control_step(wl, wl.x0, U, 5)
    assert it == 7 and len(res) == 2
    assert np.array_equal(u0, res[-1].U[0])
    assert np.array_equal(Us[:-1], res[-1].U[1:]) and np.array_equal(Us[-1], wl.u_init)


# -------------------------------------------------------------- linear-quadratic pins

def _lin(wl):
    p = wl.params
    return p["A"], p["B"], p["Q"], p["Qf"]


def test_batch_lqr_equals_riccati():
    wl = W.linear_double_integrator()
    A, B, Q, Qf = _lin(wl)
    for R in (wl.R, np.array([[0.05]]), np.array([[3.0]])):
        a = lqr.batch_lqr(A, B, Q, Qf, R, wl.dt, wl.T, wl.x0)
        b = lqr.riccati_lqr(A, B, Q, Qf, R, wl.dt, wl.T, wl.x0)
        assert np.allclose(a, b, rtol=1e-10, atol=1e-12)


def test_one_step_scalar_closed_form():
    """T = 1, scalar: x1 = x0 + beta v, S = w x1^2 + R v^2 / 2 => v* = -2 w beta x0 / (2 w beta^2 + R).
    With the coupling R = lambda / sigma one iteration lands on v* in expectation."""
    wl = W.linear_double_integrator(K=400_000, T=1, nu=3.0, lam=2.0, sigma=0.5)
    wl = wl.replace(params=dict(A=np.zeros((1, 1)), B=np.array([[1.0]]), Q=np.array([[1.0]]),
                                Qf=np.array([[2.0]])), n=1, x0=np.array([1.5]))
    beta, w, R = wl.dt, 3.0, float(wl.R[0, 0])
    v_star = -2 * w * beta * 1.5 / (2 * w * beta ** 2 + R)
    A, B, Q, Qf = _lin(wl)
    assert lqr.batch_lqr(A, B, Q, Qf, wl.R, wl.dt, 1, wl.x0)[0, 0] == pytest.approx(v_star, rel=1e-12)
    r = mppi.iteration(wl, wl.x0, np.zeros((1, 1)), 0)
    assert abs(r.U[0, 0] - v_star) < 4 * _se(r)[0, 0]
    # weighted variance of v equals the tilted variance lambda / (2 w beta^2 + R)
    var = np.sum(r.w * (r.du[:, 0, 0] - r.dU[0, 0]) ** 2)
    assert var == pytest.approx(wl.lam / (2 * w * beta ** 2 + R), rel=0.03)


@pytest.mark.parametrize("coupled", [True, False])
def test_iteration_matches_its_expectation(coupled):
    R = None if coupled else 0.3
    wl = W.linear_double_integrator(K=200_000, nu=2.0, R=R)
    A, B, Q, Qf = _lin(wl)
    U = 0.2 * np.cos(np.arange(wl.T))[:, None]
    r = mppi.iteration(wl, wl.x0, U, 1)
    ex = lqr.expected_update(A, B, Q, Qf, wl.R, wl.dt, wl.T, wl.x0, U, wl.sigma, wl.nu, wl.lam)
    assert np.max(np.abs(r.U - ex) / _se(r)) < 4.5
    lq = lqr.batch_lqr(A, B, Q, Qf, wl.R, wl.dt, wl.T, wl.x0)
    if coupled:   # one iteration reaches the LQR optimum in expectation
        assert np.allclose(ex, lq, rtol=1e-9, atol=1e-12)


def test_lqr_is_the_fixed_point_without_coupling():
    wl = W.linear_double_integrator(nu=4.0, R=0.05, lam=0.7, sigma=2.0)
    A, B, Q, Qf = _lin(wl)
    lq = lqr.batch_lqr(A, B, Q, Qf, wl.R, wl.dt, wl.T, wl.x0)
    U = np.zeros((wl.T, 1))
    for _ in range(400):
        U = lqr.expected_update(A, B, Q, Qf, wl.R, wl.dt, wl.T, wl.x0, U, wl.sigma, wl.nu, wl.lam)
    assert np.allclose(U, lq, rtol=1e-8, atol=1e-10)
    ex = lqr.expected_update(A, B, Q, Qf, wl.R, wl.dt, wl.T, wl.x0, lq, wl.sigma, wl.nu, wl.lam)
    assert np.allclose(ex, lq, rtol=1e-10, atol=1e-12)


def test_oracle_iterations_converge_to_lqr():
    wl = W.linear_double_integrator(K=100_000, nu=2.0, R=0.3)
    A, B, Q, Qf = _lin(wl)
    lq = lqr.batch_lqr(A, B, Q, Qf, wl.R, wl.dt, wl.T, wl.x0)
    U = np.zeros((wl.T, 1))
    err0 = np.abs(U - lq).max()
    for it in range(12):
        U = mppi.iteration(wl, wl.x0, U, it).U
    assert np.abs(U - lq).max() < 0.1 * err0


def test_cost_to_go_variant_equals_total_cost_when_T_is_one():
    wl = W.cartpole(K=300, T=1, nu=2.0)
    U = np.array([[0.4]])
    a = mppi.iteration(wl, wl.x0, U, 2).U
    b = mppi.iteration_cost_to_go(wl, wl.x0, U, 2)
    assert np.allclose(a, b, rtol=1e-14)


def test_closed_loop_cartpole_balances():
    """200 control steps of the cart-pole workload (nu = 2): the pole ends upright and at rest."""
    wl = W.cartpole(nu=2.0)
    x = wl.x0.copy()
    U = mppi.initial_sequence(wl)
    it = 0
    for _ in range(wl.control_steps):
        u0, U, it, _ = mppi.control_step(wl, x, U, it)
        x = mppi.plant_step(wl, x, u0)
    qd = wl.params["q_diag"]
    assert float(qd @ x ** 2) < 0.1 and abs(x[2]) < 0.1 and it == 200


def _zero_state_cost(wl):
    return wl.replace(params=dict(wl.params, Q=np.zeros((2, 2)), Qf=np.zeros((2, 2))))


def test_cost_to_go_weights_only_the_future():
    """S(tau_{i,k}) is the cost of the trajectory from time i on (Section III-C): with no
    state cost, redrawing the perturbations of steps 0 and 1 leaves the updates of steps
    2.. unchanged, and changes those of steps 0 and 1."""
    from oracle.noise import control_noise
    wl = _zero_state_cost(W.linear_double_integrator(K=64, T=6, nu=2.0))
    U = np.linspace(-0.5, 0.5, 6)[:, None]
    du = control_noise(wl.seed, 0, wl.K, wl.T, wl.sigma, wl.nu)
    du2 = du.copy()
    du2[:, :2, :] = control_noise(wl.seed + 1, 0, wl.K, 2, wl.sigma, wl.nu)
    a = mppi.iteration_cost_to_go(wl, wl.x0, U, 0, du=du)
    b = mppi.iteration_cost_to_go(wl, wl.x0, U, 0, du=du2)
    assert np.array_equal(a[2:], b[2:])
    assert np.all(a[:2] != b[:2])


def test_cost_to_go_expected_update_cancels_the_nominal():
    """Zero state cost, R = lambda Sigma^-1 and exploration nu: the weight of step i is
    exp(-sum_{j>=i} [(1 - 1/nu)/2 du_j^2 + u_j du_j] / lambda) up to a constant, and under
    du_j ~ N(0, nu) the weighted density of du_i is N(-u_i, 1) (the likelihood-ratio terms
    of Section III-C undo the exploration), so U + dU -> 0 at every step as K grows."""
    wl = _zero_state_cost(W.linear_double_integrator(K=200_000, T=4, nu=2.0, lam=1.0, sigma=1.0))
    U = np.array([[0.3], [-0.2], [0.25], [0.1]])
    out = mppi.iteration_cost_to_go(wl, wl.x0, U, 0)
    assert np.abs(out).max() < 0.015, out.ravel()


def _swingup_run(nu, steps=None, K=1000, seed=1):
    """Closed loop of the swing-up task: per control step the state's running cost and the
    pole angle."""
    wl = W.cartpole_swingup(nu=nu, K=K).replace(seed=seed)
    system = systems.make(wl)
    x, U, it, qs, th = wl.x0.copy(), mppi.initial_sequence(wl), 0, [], []
    for _ in range(wl.control_steps if steps is None else steps):
        u0, U, it, _ = mppi.control_step(wl, x, U, it, system=system)
        x = mppi.plant_step(wl, x, u0, system=system)
        qs.append(system.q(x[None])[0])
        th.append(x[2])
    return np.array(qs), np.array(th)


def test_swingup_natural_variance_never_swings_up_over_the_whole_run():
    """Section V-A over the full 10 s (500 control steps, K = 1000): with the natural variance
    (nu = 1) the pole never comes up (never within 25 degrees of upright) and the average
    running cost stays near the hanging value 2000, while a large exploration variance
    (nu = 100) brings it up within 4 s and holds it balanced through the last second."""
    q1, th1 = _swingup_run(1.0)
    q100, th100 = _swingup_run(100.0)
    print("average running cost nu=1:", q1.mean(), "nu=100:", q100.mean())
    assert np.all(np.cos(th1) > -0.9)                     # never near theta = pi
    assert q1.mean() > 1500.0
    up = np.where(np.cos(th100) < -0.9)[0]
    assert up.size and up[0] * W.SWINGUP_DT < 4.0
    assert np.all(np.cos(th100[-50:]) < -0.99) and q100[-50:].mean() < 50.0


def test_swingup_exploration_variance_speeds_up_the_swing():
    """Section V-A: the swing-up gets faster as nu grows -- over the first 4 s the average
    running cost falls monotonically across nu = 3, 30, 300."""
    costs = [_swingup_run(nu, steps=200)[0].mean() for nu in (3.0, 30.0, 300.0)]
    print("average running cost over 4 s, nu = 3, 30, 300:", costs)
    assert costs[0] > costs[1] > costs[2]


# ------------------------------------------------------------- crash indicator
def _crash_quad(obstacles, **over):
    wl = W.quadrotor(K=1, T=60, obstacles=obstacles, crash=True)
    return wl.replace(params=dict(wl.params, **over))


def test_crash_indicator_free_fall_freezes_and_charges_every_later_step():
    """Zero thrust from height h: the Euler recursion gives z_i = h - g dt^2 i (i - 1) / 2.
    C switches on at the first post-transition state below the ground (Section V-C); from
    then on the state stays put and each step adds crash_cost on top of the state cost."""
    h, g, dt, T, cc = 0.3, W.QUAD_GRAVITY, 0.01, 60, W.QUAD_CRASH_COST
    wl = _crash_quad(np.zeros((0, 4)))
    system = systems.make(wl)
    x0 = np.zeros(12)
    x0[2] = h
    U = np.zeros((T, 4))
    du = np.zeros((1, T, 4))
    seen = []
    S = mppi.rollout_costs(system, x0, U, du, dt, np.asarray(wl.R), wl.nu,
                           observer=lambda i, x: seen.append(x[0].copy()))
    z = h - g * dt * dt * np.arange(1, T + 1) * np.arange(0, T) / 2.0     # z after step i
    i_star = int(np.argmax(z < 0.0))
    assert 0 < i_star < T - 1
    zs = np.array([s[2] for s in seen])
    assert np.allclose(zs[:i_star + 1], z[:i_star + 1], atol=1e-12)
    assert np.all(zs[i_star:] == zs[i_star])                            # frozen where it crashed
    goal = np.asarray(wl.params["goal"])
    p = np.zeros((T, 3))
    p[:, 2] = np.where(np.arange(T) < i_star, z, z[i_star])
    want = np.sum(np.sum((p - goal) ** 2, axis=1)) + cc * (T - i_star)
    assert abs(S[0] - want) < 1e-9 * want


def test_crash_indicator_obstacle_hit_at_constant_velocity():
    """Hover thrust, level attitude, horizontal speed v: x_i = v dt i.  An obstacle of radius r
    at (c, 0, z0) is hit at the first step with |x_i - c| < r; with crash_cost = 0 the same
    rollout flies through, so the difference of the two path costs is crash_cost times the
    steps from the hit on plus the state-cost difference of the frozen tail."""
    v, dt, T, c, r = 2.0, 0.01, 60, 0.5, 0.2
    obs = np.array([[c, 0.0, 1.5, r]])
    wl = _crash_quad(obs, w_obs=0.0)
    on, off = systems.make(wl), systems.make(wl.replace(params=dict(wl.params, crash_cost=0.0)))
    x0 = np.zeros(12)
    x0[2], x0[3] = 1.5, v
    U = np.full((T, 4), W.QUAD_HOVER)
    du = np.zeros((1, T, 4))
    R = np.asarray(wl.R)
    S_on = mppi.rollout_costs(on, x0, U, du, dt, R, wl.nu)[0]
    S_off = mppi.rollout_costs(off, x0, U, du, dt, R, wl.nu)[0]
    xs = v * dt * np.arange(1, T + 1)
    i_star = int(np.argmax(np.abs(xs - c) < r))
    goal = np.asarray(wl.params["goal"])
    q = lambda px: (px - goal[0]) ** 2 + (0.0 - goal[1]) ** 2 + (1.5 - goal[2]) ** 2
    frozen = np.where(np.arange(T) < i_star, xs, xs[i_star])
    want = np.sum(q(frozen) - q(xs)) + W.QUAD_CRASH_COST * (T - i_star)
    assert abs((S_on - S_off) - want) < 1e-9 * abs(want)


def test_crash_indicator_off_changes_nothing():
    wl = W.quadrotor(K=64, T=30).replace(seed=4)
    a = mppi.iteration(wl, wl.x0, mppi.initial_sequence(wl), 0)
    wl0 = wl.replace(params={k: v for k, v in wl.params.items() if k not in ("crash_cost", "ground_z")})
    b = mppi.iteration(wl0, wl0.x0, mppi.initial_sequence(wl0), 0)
    assert np.array_equal(a.S, b.S)
