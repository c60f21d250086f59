"""Learned dynamics on the GPU (BF16 MFMA) through the C ABI against the FP64 oracle with
bfloat16 emulation: dataset targets and statistics, forward, loss and gradients, training,
and one MPPI iteration with the network as the rollout model."""
import numpy as np
import pytest

import paper_1509_01149_amd as P
import workloads as W
from oracle import mlp as omlp
from oracle import mppi
from tests._parity import _first_order, u_tolerance

pytestmark = pytest.mark.gpu

# Element-wise bars of the BF16 network against the BF16-emulating FP64 oracle: per element, the
# worst-case FP32 summation error of its own product plus the propagation of every bfloat16
# operand whose FP32 value can round the other way than its FP64 value (tests/_mlp_bounds.py,
# derived from the arithmetic and pinned on the CPU against an FP32 realisation and planted
# mistakes in tests/test_oracle_mlp.py).
from tests import _mlp_bounds as MB  # noqa: E402


def assert_elementwise(got, ref, bound, what):
    excess = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(ref, dtype=np.float64)) / bound
    print(what, "worst |d| / bound", float(excess.max()))
    assert np.all(excess <= 1.0), (what, float(excess.max()))


def _stats_net(seed=5, n=20000):
    wl = W.quadrotor()
    x, u = W.mlp_training_inputs(n)
    d = omlp.transitions(wl, x, u)
    z = np.concatenate([x, u], 1)
    st = omlp.standardisation(z, d)
    w = W.mlp_init_weights(seed)
    net = omlp.Net(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], *st)
    return wl, x, u, d, net, w


def _stats_vec(net):
    return np.concatenate([net.mu_in, net.sd_in, net.mu_out, net.sd_out])


def test_dataset_targets_and_statistics():
    wl, x, u, d, net, w = _stats_net()
    g = P.Mlp(w)
    g.set_dataset(wl.params, wl.dt, x, u)
    td = g.targets()
    assert np.max(np.abs(td - d) / np.maximum(1e-3, np.abs(d))) < 1e-6
    assert np.allclose(g.stats(), _stats_vec(net), rtol=1e-6, atol=1e-9)


def test_forward_matches_bf16_oracle():
    wl, x, u, d, net, w = _stats_net()
    rng = np.random.default_rng(1)
    net.b1 += 0.1 * rng.standard_normal(128)
    net.b2 += 0.1 * rng.standard_normal(128)
    net.b3 += 0.1 * rng.standard_normal(12)
    g = P.Mlp(dict(W1=net.W1, b1=net.b1, W2=net.W2, b2=net.b2, W3=net.W3, b3=net.b3))
    g.set_stats(_stats_vec(net))
    B = 3000     # ragged against the 32-row GEMM tiles
    dx_g = g.forward(x[:B], u[:B])
    dx_o = omlp.predict_delta(net, x[:B], u[:B], bf16=True)
    yg, yo = (dx_g - net.mu_out) / net.sd_out, (dx_o - net.mu_out) / net.sd_out
    err = np.abs(yg - yo)
    print("forward: max", err.max(), "mean", err.mean())
    z = np.concatenate([x[:B], u[:B]], 1)
    bound, _ = MB.forward_bounds(net, (z - net.mu_in) / net.sd_in)
    assert_elementwise(yg, yo, bound, "forward (standardised outputs)")


@pytest.mark.parametrize("B", [48, 4096])
def test_gradients_match_bf16_oracle(B):
    """Every element of every gradient, at a small ragged batch (one product per tile, tight
    summation bounds) and at a full minibatch (the split-K path over the batch)."""
    wl, x, u, d, net, w = _stats_net()
    z = np.concatenate([x, u], 1)
    zn = (z - net.mu_in) / net.sd_in
    tn = (d - net.mu_out) / net.sd_out
    g = P.Mlp(w)
    loss_g, grads_g = g.loss_grads(zn[:B], tn[:B])
    loss_o, grads_o = omlp.loss_and_grads(net, omlp.bf16_round(zn[:B]), tn[:B], bf16=True)
    assert loss_g == pytest.approx(loss_o, rel=1e-4)
    bounds = MB.gradient_bounds(net, zn[:B], tn[:B])
    for (k, _), go, bd in zip(P.binding._MLP_SHAPES, grads_o, bounds):
        assert_elementwise(grads_g[k], go, bd, "gradient " + k)


def test_training_tracks_the_oracle():
    wl, x, u, d, net, w = _stats_net(n=16384)
    g = P.Mlp(w)
    g.set_dataset(wl.params, wl.dt, x, u)
    order = np.concatenate(W.minibatch_order(16384, 3))
    losses_g = g.train(order, 1024, 2e-3)
    z = np.concatenate([x, u], 1)
    zn = omlp.bf16_round((z - net.mu_in) / net.sd_in)
    tn = (d - net.mu_out) / net.sd_out
    opt = omlp.Adam(net, lr=2e-3)
    losses_o = []
    for s in range(len(losses_g)):
        idx = order[s * 1024:(s + 1) * 1024]
        l, gr = omlp.loss_and_grads(net, zn[idx], tn[idx], bf16=True)
        losses_o.append(l)
        opt.step(net, gr)
    losses_o = np.array(losses_o)
    print("losses gpu", losses_g[[0, 10, -1]], "oracle", losses_o[[0, 10, -1]])
    assert losses_g[-1] < 0.3 * losses_g[0]
    assert np.allclose(losses_g, losses_o, rtol=0.05)


def test_mppi_iteration_with_learned_dynamics():
    wl0, x, u, d, net, w = _stats_net()
    rng = np.random.default_rng(2)
    g = P.Mlp(w)
    g.set_stats(_stats_vec(net))
    wl = W.quadrotor_mlp(g, nu=2.0, K=4096 + 37, T=50).replace(seed=9)
    sysm = omlp.QuadrotorMLP(wl.params, net, bf16=True)
    U0 = mppi.initial_sequence(wl)
    with P.controller_for(wl) as c:
        u0 = c.step(wl.x0)
        U = c.get_controls()
        S_gpu, rho, eta, dU = c.debug_last()
    u0_r, U_r, _, res = mppi.control_step(wl, wl.x0, U0, 0, system=sysm)
    S = res[-1].S
    rel = np.abs(S_gpu - S) / np.maximum(1.0, np.abs(S))
    scale = max(1.0, float(np.max(np.abs(U_r))), float(np.max(np.abs(u0_r))))
    fin = np.isfinite(S) & np.isfinite(S_gpu)
    m = dict(u0_err=float(np.max(np.abs(u0[:wl.m] - u0_r))) / scale, U_err=float(np.max(np.abs(U - U_r))) / scale,
             first_order=float(np.max(np.abs(_first_order(res[-1], S_gpu, fin, wl.lam)))) / scale)
    tol, met = u_tolerance(m)
    print("mlp mppi: S rel max", rel.max(), "median", np.median(rel), "U", m["U_err"], met)
    assert np.median(rel) < 1e-4 and rel.max() < 1e-2
    assert m["U_err"] <= tol and m["u0_err"] <= tol


def test_trained_network_gain_over_untrained_and_against_analytic():
    """Train on 1e6 analytic transitions on the GPU, then assess the learned model against
    the analytic one: one-step error on held-out transitions, open-loop trajectory error,
    control error of one MPPI iteration, and closed-loop cost on the analytic plant
    against (a) MPPI with the analytic model and (b) MPPI with the untrained network."""
    from oracle import systems
    wl = W.quadrotor()
    x, u = W.mlp_training_inputs(1_000_000)
    init = W.mlp_init_weights()
    g = P.Mlp(init)
    g.set_dataset(wl.params, wl.dt, x, u)
    stats = g.stats()
    epochs = 20
    for ep, order in enumerate(W.minibatch_order(1_000_000, epochs)):
        losses = g.train(order, 4096, 2e-3 * 0.5 ** (ep // 5))
    assert losses.mean() < 1e-3
    xh, uh = W.mlp_training_inputs(20000, seed=999)
    nrmse = np.sqrt(np.mean(((g.forward(xh, uh) - omlp.transitions(wl, xh, uh)) / stats[44:56]) ** 2, 0))
    assert nrmse.max() < 0.05, nrmse
    untrained = P.Mlp(init)
    untrained.set_stats(stats)
    sysa = systems.make(wl)

    def closed_loop(model, steps=150, K=4096):
        w = (W.quadrotor(nu=2.0, K=K, T=100) if model is None else W.quadrotor_mlp(model, nu=2.0, K=K, T=100))
        w = w.replace(seed=3)
        xs, cost = w.x0.copy(), 0.0
        with P.controller_for(w) as c:
            for _ in range(steps):
                xs = mppi.plant_step(wl, xs, c.step(xs))
                cost += float(sysa.q(xs[None])[0])
        return cost

    c_ana, c_trained, c_untrained = closed_loop(None), closed_loop(g), closed_loop(untrained)
    print("closed-loop cost: analytic", c_ana, "trained", c_trained, "untrained", c_untrained)
    assert c_trained < 0.85 * c_untrained          # what training gains
    assert c_trained < 1.25 * c_ana                # and how close it comes to the analytic model
    wa = W.quadrotor(nu=2.0, K=16384, T=100).replace(seed=5)
    wm = W.quadrotor_mlp(g, nu=2.0, K=16384, T=100).replace(seed=5)
    with P.controller_for(wa) as ca:
        ca.step(wa.x0)
        Ua = ca.get_controls()
    with P.controller_for(wm) as cm:
        cm.step(wm.x0)
        Um = cm.get_controls()
    ctrl_err = float(np.max(np.abs(Um - Ua)) / np.max(np.abs(Ua)))
    xa, xm = wa.x0.copy(), wa.x0.copy()
    for i in range(100):
        xa = mppi.plant_step(wa, xa, Ua[i])
        xm = xm + g.forward(xm[None], Ua[i][None])[0]
    traj_err = float(np.linalg.norm(xa[:3] - xm[:3]))
    print("control error (rel)", ctrl_err, "trajectory position error after 100 steps", traj_err)
    assert ctrl_err < 0.01 and traj_err < 0.3
