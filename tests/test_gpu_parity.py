"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs, for every compiled-in system at the workloads' full sizes, plus the edge cases
(one sample, ragged sample counts, one-step horizons, horizons that leave a partial
noise group, zero noise)."""
import numpy as np
import pytest

import paper_1509_01149_amd as P
import workloads as W
from oracle import mppi, noise, philox, systems
from tests._parity import _first_order, assert_parity, controller, one_step

pytestmark = pytest.mark.gpu


def test_philox_bits_match_oracle():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    for seed in (0, 0xDEADBEEF12345678, 1 << 40):
        out = P.philox(ctr, seed)
        ref = np.stack(philox.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3],
                                            seed & 0xFFFFFFFF, seed >> 32), axis=1)
        assert np.array_equal(out, ref)


@pytest.mark.parametrize("G", [4, 16, 32])
def test_lane_group_primitives(G):
    """The DPP and swizzle scans, broadcasts and sums the step-split rollouts are built on,
    against their definitions.  Small integers (and slopes in {1, -1, 2}) keep every sum
    and product exact in FP32, so the comparison is bitwise."""
    rng = np.random.default_rng(G)
    n = 3 * 64
    a = rng.integers(-8, 9, size=n).astype(np.float32)
    b = rng.integers(-8, 9, size=n).astype(np.float32)
    out = P.binding.lane_groups(a, b, G)
    ag = a.reshape(-1, G)
    incl = np.cumsum(ag, axis=1)
    assert np.array_equal(out[:, 0], incl.ravel())
    assert np.array_equal(out[:, 1], (incl - ag).ravel())
    assert np.array_equal(out[:, 2], np.repeat(ag[:, -1], G))
    assert np.array_equal(out[::G, 3], ag.sum(axis=1))
    slope = rng.choice(np.array([1.0, -1.0, 2.0], dtype=np.float32), size=n)
    out = P.binding.lane_groups(slope, b, G)
    if G > 16:
        assert np.all(np.isnan(out[:, 4:]))
        return
    ref = np.zeros((n, 2), dtype=np.float64)
    for g0 in range(0, n, G):
        A, B = 1.0, 0.0
        for t in range(g0, g0 + G):                  # lane t's map after those before it
            A, B = slope[t] * A, slope[t] * B + b[t]
            ref[t] = A, B
    assert np.array_equal(out[:, 4:].astype(np.float64), ref)


@pytest.mark.parametrize("T,m", [(100, 1), (7, 2), (150, 4)])
def test_normals_match_oracle(T, m):
    wl = {1: W.cartpole(K=64, T=T), 2: W.bicycle(K=64, T=T), 4: W.quadrotor(K=64, T=T)}[m].replace(seed=77)
    with controller(wl) as c:
        it = (1 << 32) + 3
        g = c.debug_normals(it, 100, 300)
        ref = noise.standard_normals(77, it, 300, T, m, k_offset=100)
        err = np.abs(g - ref) / np.maximum(1.0, np.abs(ref))
        assert err.max() < 2e-6, err.max()


CASES = {
    "cartpole_nu1": lambda: W.cartpole(nu=1.0),
    "cartpole_nu2": lambda: W.cartpole(nu=2.0),
    "bicycle": lambda: W.bicycle(),
    "quadrotor_nu1": lambda: W.quadrotor(nu=1.0),
    "quadrotor_nu2": lambda: W.quadrotor(nu=2.0),
    "quadrotor_nu4": lambda: W.quadrotor(nu=4.0),
    "linear": lambda: W.linear_double_integrator(K=4096, R=0.3),
    # per-dimension exploration factors, A = diag(sqrt(nu_j))
    "quadrotor_nu_diag": lambda: W.quadrotor(nu=np.array([1.0, 2.0, 4.0, 8.0]), lam=420.0),
    "bicycle_nu_diag": lambda: W.bicycle(nu=np.array([1.0, 4.0])),
    # the swing-up task of Section V-A (velocity-command cart, pole hanging at rest)
    "swingup_nu1": lambda: W.cartpole_swingup(nu=1.0),
    "swingup_nu1000": lambda: W.cartpole_swingup(nu=1000.0, K=4096),
    # step-split lane counts: K above 8192 takes 4 lanes per sample (ragged horizon, last
    # chunk partial); K = 8192 is the largest with 16; the bicycle takes 32 up to K = 4096
    # (the default cases; here also a partial last block and a single ragged chunk)
    "bicycle_4lanes": lambda: W.bicycle(K=9000, T=37),
    "bicycle_16lanes_k8192": lambda: W.bicycle(K=8192, T=100),
    "bicycle_32lanes_ragged": lambda: W.bicycle(K=4000, T=37),
    # obstacle counts around the 32 the quad holds in registers: 100 (the rest read from LDS
    # each step), 5 (most register slots empty), none; and spheres large enough that the
    # obstacle scale (a power of two with s (r + margin)^2 <= 1/4) is 2^-8
    "quadrotor_100_obstacles": lambda: W.quadrotor(K=2048, T=100, obstacles=W.obstacle_field(n=100)),
    "quadrotor_5_obstacles": lambda: W.quadrotor(K=2048, T=100, obstacles=W.obstacle_field(n=5)),
    "quadrotor_no_obstacles": lambda: W.quadrotor(K=2048, T=60, obstacles=np.zeros((0, 4))),
    "quadrotor_large_obstacles": lambda: W.quadrotor(K=2048, T=100, obstacles=np.array(
        [[4.0, 3.5, 1.5, 2.5], [4.0, -4.0, 1.0, 3.0], [9.0, 8.0, 2.0, 6.5]])),
}


@pytest.mark.parametrize("name", list(CASES))
def test_first_iteration_parity(name):
    wl = CASES[name]().replace(seed=3)
    U0 = mppi.initial_sequence(wl)
    with controller(wl) as c:
        assert c.info()["rollout_mode"] & P.binding.ROLLOUT_DIAGONAL    # diagonal Sigma and R here
        m = one_step(wl, c, wl.x0, U0, 0)
    print(name, {k: v for k, v in m.items() if isinstance(v, (float, int, bool))})
    assert_parity(m, label=name)


def full_sigma_cases():
    """Full (non-diagonal) SPD covariances, so the rollouts take the general products: a
    lower-triangular A chol(Sigma) for the perturbations and a full likelihood-ratio matrix.
    `coupled` passes R = NULL to the library (R = lambda Sigma^-1 formed there) and the same
    matrix explicitly to the oracle."""
    sb = np.array([[0.5, 0.1], [0.1, 0.3]])
    sq = 0.2 * np.eye(4) + 0.05 * np.ones((4, 4))
    return {
        "bicycle_coupled": (W.bicycle().replace(sigma=sb, R=130.0 * np.linalg.inv(sb)), True),
        "bicycle_coupled_nu_diag": (W.bicycle(nu=np.array([1.0, 4.0])).replace(sigma=sb, R=130.0 * np.linalg.inv(sb)),
                                    True),
        "bicycle_decoupled_16lanes": (W.bicycle(K=8000, T=50).replace(sigma=sb), False),
        "quadrotor_decoupled": (W.quadrotor(nu=2.0, K=4096, T=150).replace(sigma=sq), False),
        "quadrotor_coupled": (W.quadrotor(nu=2.0, K=4096, T=100).replace(sigma=sq, R=420.0 * np.linalg.inv(sq)), True),
        "quadrotor_nu_diag": (W.quadrotor(nu=np.array([1.0, 2.0, 4.0, 8.0]), lam=420.0, K=2048, T=150)
                              .replace(sigma=sq), False),
    }


@pytest.mark.parametrize("name", list(full_sigma_cases()))
def test_full_covariance_parity(name):
    wl, coupled = full_sigma_cases()[name]
    wl = wl.replace(seed=19)
    with controller(wl, **(dict(R=None) if coupled else {})) as c:
        info = c.info()
        assert not info["rollout_mode"] & P.binding.ROLLOUT_DIAGONAL, info
        m = one_step(wl, c, wl.x0, mppi.initial_sequence(wl), 0)
    assert_parity(m, label=name)


@pytest.mark.parametrize("name", ["bicycle", "quadrotor_nu2", "swingup_nu1000"])
def test_warm_started_steps_parity(name):
    """Several control steps; before each the oracle is given the GPU's own nominal
    sequence and state, so only one step's arithmetic is compared at a time."""
    wl = CASES[name]().replace(seed=5, n_iters=2)
    x = wl.x0.copy()
    it = 0
    with controller(wl) as c:
        for step in range(3):
            U_before = c.get_controls()
            m = one_step(wl, c, x, U_before, it, n_iters=2)
            assert_parity(m)
            it = m["iteration"]
            x = mppi.plant_step(wl, x, m["u0_gpu"])


def test_closed_loop_cartpole_per_step():
    """The 200-step cart-pole run, with the oracle re-seeded from the GPU each step."""
    wl = W.cartpole(nu=2.0).replace(seed=1)
    x = wl.x0.copy()
    worst = 0.0
    conditioned = 0
    with controller(wl) as c:
        for step in range(wl.control_steps):
            U_before = c.get_controls()
            m = one_step(wl, c, x, U_before, step)
            assert_parity(m)
            worst = max(worst, m["U_err"])
            conditioned += m["U_err"] > 1e-4
            x = mppi.plant_step(wl, x, m["u0_gpu"])
    print("closed-loop worst U_err", worst, "steps beyond 1e-4 (explained to first order):", conditioned,
          "final x", x)
    assert conditioned <= 20
    assert abs(x[2]) < 0.2


@pytest.mark.parametrize("K,T", [(1, 10), (257, 7), (1000, 1), (4097, 13), (300, 3)])
def test_ragged_and_tiny_shapes(K, T):
    for wl in (W.bicycle(K=K, T=T), W.cartpole(nu=2.0, K=K, T=T), W.quadrotor(K=K, T=T)):
        wl = wl.replace(seed=11)
        with controller(wl) as c:
            m = one_step(wl, c, wl.x0, mppi.initial_sequence(wl), 0)
        assert_parity(m)


def test_zero_noise_only_shifts():
    wl = W.cartpole(K=300, T=20).replace(sigma=np.zeros((1, 1)), R=np.array([[0.01]]))
    U = np.linspace(-1, 1, 20)[:, None]
    with controller(wl, u_nominal0=U) as c:
        u0 = c.step(wl.x0)
        assert u0[0] == U[0, 0]
        assert np.array_equal(c.get_controls(), np.vstack([U[1:], [[0.0]]]))


def test_linear_small_state():
    """n = 2 < 4: the linear system must not touch state words beyond n."""
    wl = W.linear_double_integrator(K=2048, R=0.3).replace(seed=2)
    with controller(wl) as c:
        m = one_step(wl, c, wl.x0, mppi.initial_sequence(wl), 0)
    assert_parity(m)


def test_fused_plant_step_equals_step_then_plant():
    """mppi_step_plant_async == mppi_step_async + mppi_plant_step_async, bitwise; and the
    device plant agrees with the oracle's FP64 plant step."""
    import torch
    for wl in (W.bicycle(K=2048, T=50), W.quadrotor(nu=2.0, K=1024, T=60), W.cartpole(nu=2.0)):
        wl = wl.replace(seed=13)
        dev = torch.device("cuda:0")
        xa = torch.tensor(wl.x0, dtype=torch.float64, device=dev)
        xb = xa.clone()
        ua = torch.zeros(wl.m, dtype=torch.float64, device=dev)
        ub = ua.clone()
        with controller(wl) as a, controller(wl) as b:
            for _ in range(5):
                x_before = xb.cpu().numpy()
                a.step_plant_async(xa.data_ptr(), ua.data_ptr())
                b.step_async(xb.data_ptr(), ub.data_ptr())
                b.plant_step_async(xb.data_ptr(), ub.data_ptr())
                a.sync()
                b.sync()
                x_ref = mppi.plant_step(wl, x_before, ub.cpu().numpy())
                assert np.allclose(xb.cpu().numpy(), x_ref, rtol=1e-12, atol=1e-12)
            assert torch.equal(xa, xb) and torch.equal(ua, ub)
            assert np.array_equal(a.get_controls(), b.get_controls())


CTG_CASES = {
    "linear": lambda: W.linear_double_integrator(K=4096, T=20, R=0.3),
    "bicycle": lambda: W.bicycle(K=4096, T=100),
    "bicycle_nu_diag": lambda: W.bicycle(K=3000, T=37, nu=np.array([1.0, 4.0])),
    "bicycle_4lanes": lambda: W.bicycle(K=9000, T=37),
    # running costs beyond the rollout block's 32 KiB: the separate per-step minimum pass
    "bicycle_long_horizon": lambda: W.bicycle(K=4096, T=600),
    "quadrotor": lambda: W.quadrotor(nu=2.0, K=4096, T=60),
}


@pytest.mark.parametrize("name", list(CTG_CASES))
def test_cost_to_go_parity(name):
    """Cost-to-go weighting: step i weighted by each sample's cost from step i on, with its
    own minimum and normaliser, against the oracle's per-step softmax of tail sums."""
    wl = CTG_CASES[name]().replace(seed=7)
    U0 = mppi.initial_sequence(wl) + 0.1 * np.sin(np.arange(wl.T))[:, None]
    with controller(wl, u_nominal0=U0, weighting=P.WEIGHT_COST_TO_GO) as c:
        u0 = c.step(wl.x0)
        U_gpu = np.vstack([u0[None, :], c.get_controls()[:-1]])
        S_gpu = c.debug_last()[0]
    U_orc = mppi.iteration_cost_to_go(wl, wl.x0, U0, 0)
    S_orc = mppi.iteration(wl, wl.x0, U0, 0).S
    scale = max(1.0, np.abs(U_orc).max())
    err = np.abs(U_gpu - U_orc).max() / scale
    s_err = (np.abs(S_gpu - S_orc) / np.maximum(1.0, np.abs(S_orc))).max()
    print(name, "U err", err, "S err", s_err)
    assert s_err <= 4e-4
    assert err <= 1e-4, err


def test_cost_to_go_first_step_equals_path_weighting():
    """At step 0 the cost-to-go is the whole path cost: u_0 must be bitwise the same under
    both weightings through the same kernels (three per iteration, or two: the fused
    iterations weight step 0 against the same block minima), and the same to FP64
    reassociation across the two kernel counts; later steps must differ."""
    wl = W.bicycle(K=2048, T=50).replace(seed=9)
    ctg = P.WEIGHT_COST_TO_GO
    with controller(wl, kernels=P.KERNELS_THREE) as a, controller(wl, weighting=ctg, kernels=P.KERNELS_THREE) as b, \
            controller(wl, kernels=P.KERNELS_FUSED) as f, controller(wl, weighting=ctg, kernels=P.KERNELS_FUSED) as g:
        assert g.info()["rollout_mode"] & P.binding.ROLLOUT_FUSED
        ua, ub, uf, ug = a.step(wl.x0), b.step(wl.x0), f.step(wl.x0), g.step(wl.x0)
        assert np.array_equal(ua, ub)
        assert np.array_equal(uf, ug)
        assert np.max(np.abs(uf - ub)) <= 1e-9 * max(1.0, np.max(np.abs(ub)))
        assert not np.array_equal(a.get_controls(), b.get_controls())
        assert not np.array_equal(f.get_controls(), g.get_controls())


def test_swingup_closed_loop_exploration_variance():
    """Section V-A: 10 s of swing-up (500 control steps, K = 1000) on the GPU path, the
    plant stepped by the oracle's FP64 model.  The natural variance (nu = 1) never brings the
    pole up and its average running cost stays near the hanging value 2000; nu = 1000 brings
    it up within 4 s and keeps it balanced through the last second."""
    avg, th = {}, {}
    for nu in (1.0, 1000.0):
        wl = W.cartpole_swingup(nu=nu).replace(seed=1)
        sysm = systems.make(wl)
        x, qs, ths = wl.x0.copy(), [], []
        with controller(wl) as c:
            for _ in range(wl.control_steps):
                x = mppi.plant_step(wl, x, c.step(x), system=sysm)
                qs.append(float(sysm.q(x[None])[0]))
                ths.append(x[2])
        avg[nu], th[nu] = float(np.mean(qs)), np.array(ths)
        print("nu", nu, "average running cost", avg[nu], "final state", x)
    assert np.all(np.cos(th[1.0]) > -0.9) and avg[1.0] > 1500.0
    up = np.where(np.cos(th[1000.0]) < -0.9)[0]
    assert up.size and up[0] * wl.dt < 4.0 and np.all(np.cos(th[1000.0][-50:]) < -0.99)
    assert avg[1.0] > 2.0 * avg[1000.0]


@pytest.mark.parametrize("T,margin", [(100, 0.1), (150, 0.1), (150, 0.0)])
def test_crash_indicator_parity(T, margin):
    """Quadrotor with the crash indicator (Section V-C).  The indicator is a threshold on
    the FP32 state, so a sample grazing the ground or an obstacle may crash one step earlier
    or later than in the FP64 oracle: such a flip changes its cost by about crash_cost per
    step.  Flips must be rare (<= 0.5 % of samples); every other sample meets the usual
    per-sample cost tolerance; the update meets the usual bar plus what the flipped samples'
    weights can move it (sum of their weights on either side times max |du|).  With no
    safety margin the barrier and the obstacle coincide: every obstacle's crash threshold on
    the barrier argument is zero."""
    wl = W.quadrotor(nu=2.0, K=4096, T=T, crash=True).replace(seed=3)
    wl = wl.replace(params=dict(wl.params, obs_margin=margin))
    U0 = mppi.initial_sequence(wl)
    with controller(wl) as c:
        m = one_step(wl, c, wl.x0, U0, 0)
    last = m["res"][-1]
    S_gpu, S_orc = m["S_gpu"], last.S
    fin = np.isfinite(S_orc) & np.isfinite(S_gpu)
    flip = fin & (np.abs(S_gpu - S_orc) > 0.5 * W.QUAD_CRASH_COST)
    rel = np.abs(S_gpu - S_orc) / np.maximum(1.0, np.abs(S_orc))
    ok = fin & ~flip
    print("T", T, "flips", int(flip.sum()), "S err (others)", rel[ok].max(), "U err", m["U_err"])
    assert flip.sum() <= 0.005 * wl.K
    assert rel[ok].max() <= 4e-4
    w_gpu, _, _, _, _ = mppi.weights_and_update(np.where(np.isfinite(S_gpu), S_gpu, np.inf), last.du, wl.lam)
    moved = float(np.sum(last.w[flip]) + np.sum(w_gpu[flip])) * float(np.abs(last.du).max())
    scale = max(1.0, np.abs(U0).max())
    first = float(np.max(np.abs(_first_order(last, S_gpu, ok, wl.lam)))) / scale
    assert m["U_err"] <= 1e-4 + 2.0 * first + moved / scale
    assert m["stage_err"] <= 1e-5


def test_all_costs_non_finite_leaves_the_sequence_and_reports():
    """Every sample's path cost overflows FP32 (state cost ~1e60): the iteration leaves U
    unchanged, the step still emits u0 and shifts, MPPI_ENUMERIC is reported, and the
    controller recovers on the next finite step."""
    wl = W.linear_double_integrator(K=1000, T=10, R=0.3).replace(seed=31)
    U = np.linspace(-0.5, 0.5, wl.T)[:, None]
    with controller(wl, u_nominal0=U) as c:
        with pytest.raises(P.NumericError):
            c.step(np.array([1e30, 0.0]))
        assert np.array_equal(c.get_controls(), np.vstack([U[1:], [[0.0]]]))
        assert c.iteration() == 1
        S, rho, eta, dU = c.debug_last()
        assert np.all(np.isinf(S)) and np.all(dU == 0.0)
        U1 = c.get_controls()
        c.step(wl.x0)                                          # finite again
        m_res = mppi.control_step(wl, wl.x0, U1, 1)
        assert np.abs(c.get_controls() - m_res[1]).max() < 1e-4


def test_graph_cache_stays_bounded_and_correct():
    """Steps with many different device buffers (one captured graph each) past the cache
    bound give the same controls as one buffer reused."""
    import torch
    wl = W.bicycle(K=1024, T=20).replace(seed=33)
    dev = torch.device("cuda:0")
    with controller(wl) as a, controller(wl) as b:
        xs = [torch.tensor(wl.x0, dtype=torch.float64, device=dev) for _ in range(20)]
        us = [torch.zeros(wl.m, dtype=torch.float64, device=dev) for _ in range(20)]
        x_one = torch.tensor(wl.x0, dtype=torch.float64, device=dev)
        u_one = torch.zeros(wl.m, dtype=torch.float64, device=dev)
        for j in range(20):
            a.step_async(xs[j].data_ptr(), us[j].data_ptr())
            b.step_async(x_one.data_ptr(), u_one.data_ptr())
            a.sync()
            b.sync()
            assert torch.equal(us[j], u_one)
        assert np.array_equal(a.get_controls(), b.get_controls())


def test_closed_loop_run_equals_single_steps():
    """mppi_run_closed_loop_async over n steps == n calls of mppi_step_plant_async, bitwise:
    the captured run and the single steps launch the same kernels (the finalize with the
    plant step fused); both weightings, so both the two- and the three-kernel iteration."""
    import torch
    dev = torch.device("cuda:0")
    cases = [(W.bicycle(K=2048, T=50), P.WEIGHT_PATH), (W.quadrotor(nu=2.0, K=1024, T=40), P.WEIGHT_PATH),
             (W.cartpole(nu=2.0), P.WEIGHT_PATH), (W.bicycle(K=2048, T=50), P.WEIGHT_COST_TO_GO),
             (W.linear_double_integrator(K=1000, T=30, R=0.3), P.WEIGHT_PATH),
             (W.cartpole_swingup(nu=1000.0, K=1024, T=50), P.WEIGHT_PATH)]
    for wl, weighting in cases:
        wl = wl.replace(seed=37)
        xa = torch.tensor(wl.x0, dtype=torch.float64, device=dev)
        xb = xa.clone()
        log = torch.zeros((7, wl.m), dtype=torch.float64, device=dev)
        ub = torch.zeros((7, wl.m), dtype=torch.float64, device=dev)
        with controller(wl, weighting=weighting) as a, controller(wl, weighting=weighting) as b:
            a.run_closed_loop_async(xa.data_ptr(), 7, log.data_ptr())
            for j in range(7):
                b.step_plant_async(xb.data_ptr(), ub[j].data_ptr())
            a.sync()
            b.sync()
            assert torch.equal(xa, xb) and torch.equal(log, ub)
            assert np.array_equal(a.get_controls(), b.get_controls()) and a.iteration() == b.iteration() == 7
