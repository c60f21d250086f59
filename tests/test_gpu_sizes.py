"""Parity at the full and the maximum sizes the library accepts.

* Full size, learned dynamics (K = 16384, T = 100, the configuration the bench times):
  the oracle cannot afford all 16384 BF16-emulated rollouts in a test, so it computes 64
  sampled samples one by one (spread over the first, middle and last rollout blocks), and
  the update is checked by stage isolation (the GPU's own costs through the oracle's FP64
  weights and update, with the oracle's noise for all samples).
* Maximum horizon: T = 1024 with m = 4 (T m = 4096, the finalize's limit), linear system.
* Maximum sample count: K = 2^22 (the create-time limit), full parity.
"""
import numpy as np
import pytest

import paper_1509_01149_amd as P
import workloads as W
from oracle import mlp as omlp
from oracle import mppi
from oracle.noise import control_noise
from tests._parity import assert_parity, controller, one_step

pytestmark = pytest.mark.gpu


def test_learned_dynamics_full_size_sampled():
    wl0 = W.quadrotor()
    x, u = W.mlp_training_inputs(20000)
    d = omlp.transitions(wl0, x, u)
    st = omlp.standardisation(np.concatenate([x, u], 1), d)
    w = W.mlp_init_weights(5)
    net = omlp.Net(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], *st)
    g = P.Mlp(w)
    g.set_stats(np.concatenate([net.mu_in, net.sd_in, net.mu_out, net.sd_out]))
    wl = W.quadrotor_mlp(g, nu=2.0, K=16384, T=100).replace(seed=21)
    U0 = mppi.initial_sequence(wl)
    with P.controller_for(wl) as c:
        c.step(wl.x0)
        S_gpu, rho_gpu, eta_gpu, dU_gpu = c.debug_last()
    rng = np.random.default_rng(0)
    ks = np.unique(np.concatenate([np.arange(8), wl.K // 2 + np.arange(8), wl.K - 8 + np.arange(8),
                                   rng.choice(wl.K, 40, replace=False)]))
    du_s = np.concatenate([control_noise(wl.seed, 0, 1, wl.T, wl.sigma, wl.nu, k_offset=int(k)) for k in ks])
    sysm = omlp.QuadrotorMLP(wl.params, net, bf16=True)
    S_s = mppi.rollout_costs(sysm, wl.x0, U0, du_s, wl.dt, np.asarray(wl.R), wl.nu)
    rel = np.abs(S_gpu[ks] - S_s) / np.maximum(1.0, np.abs(S_s))
    print("sampled S rel: median", np.median(rel), "max", rel.max(), "n", len(ks))
    assert np.median(rel) < 1e-4 and rel.max() < 1e-2
    du = control_noise(wl.seed, 0, wl.K, wl.T, wl.sigma, wl.nu)
    _, eta_i, rho_i, dU_i, status = mppi.weights_and_update(np.where(np.isfinite(S_gpu), S_gpu, np.inf), du, wl.lam)
    assert status == 0
    assert rho_gpu == rho_i
    assert abs(eta_gpu - eta_i) <= 1e-12 * eta_i
    assert np.max(np.abs(dU_gpu - dU_i)) <= 1e-5 * np.max(np.abs(dU_i))


def test_maximum_horizon():
    """T m = 4096: the longest sequence the finalize holds (T = 1024 steps of a 4-input
    linear system: a horizon that long would take the quadrotor's rollouts through its
    attitude singularity and to overflow, which tests FP32 range, not the kernels)."""
    base = W.linear_double_integrator(K=256, T=1024, lam=20.0)
    wl = base.replace(n=4, m=4, sigma=np.eye(4), R=0.3 * np.eye(4), u_init=np.zeros(4), x0=np.ones(4),
                      params=dict(A=-0.1 * np.eye(4), B=0.1 * np.eye(4), Q=0.01 * np.eye(4), Qf=np.eye(4)),
                      seed=23)
    with controller(wl) as c:
        m = one_step(wl, c, wl.x0, mppi.initial_sequence(wl), 0)
    print({k: v for k, v in m.items() if isinstance(v, (float, int, bool))})
    assert_parity(m)


def test_maximum_sample_count():
    """K = 2^22 (65,536 rollout blocks, 16,384 update chunks), cart-pole with a short horizon."""
    wl = W.cartpole(nu=2.0, K=1 << 22, T=4).replace(seed=29)
    with controller(wl) as c:
        m = one_step(wl, c, wl.x0, mppi.initial_sequence(wl), 0)
    print({k: v for k, v in m.items() if isinstance(v, (float, int, bool))})
    assert_parity(m)
