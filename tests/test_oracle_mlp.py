"""Pins of the oracle's learned-dynamics MLP (CPU only), against independent
implementations: torch's CPU bfloat16 conversion, torch autograd for the gradients,
torch.optim.Adam for the optimiser, and central finite differences."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import mlp


def _net(seed=5):
    w = W.mlp_init_weights(seed)
    rng = np.random.default_rng(seed)
    b1, b2, b3 = (0.1 * rng.standard_normal(n) for n in (128, 128, 12))
    return mlp.Net(w["W1"], b1, w["W2"], b2, w["W3"], b3, rng.standard_normal(16), rng.uniform(0.5, 2, 16),
                   rng.standard_normal(12), rng.uniform(0.1, 1, 12))


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def _torch_forward(net, zn, bf16):
    t = lambda a: torch.tensor(a, dtype=torch.float64)
    r = (lambda a: a.to(torch.float32).to(torch.bfloat16).to(torch.float64)) if bf16 else (lambda a: a)
    W1, b1, W2, b2, W3, b3 = (t(p).requires_grad_(True) for p in net.params())
    h1 = torch.tanh(r(t(zn)) @ r(W1).T + b1)
    h2 = torch.tanh(r(h1) @ r(W2).T + b2)
    y = r(h2) @ r(W3).T + b3
    return y, [W1, b1, W2, b2, W3, b3]


def test_forward_matches_torch():
    net = _net()
    zn = np.random.default_rng(1).standard_normal((64, 16))
    for bf16 in (False, True):
        y, _ = mlp.forward_normalised(net, zn, bf16)
        yt, _ = _torch_forward(net, zn, bf16)
        assert np.allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_gradients_match_autograd_and_finite_differences():
    net = _net()
    rng = np.random.default_rng(2)
    zn, tn = rng.standard_normal((32, 16)), rng.standard_normal((32, 12))
    loss, g = mlp.loss_and_grads(net, zn, tn)
    y, ps = _torch_forward(net, zn, False)
    lt = torch.mean((y - torch.tensor(tn)) ** 2)
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-13)
    for gi, p in zip(g, ps):
        assert np.allclose(gi, p.grad.numpy(), rtol=1e-10, atol=1e-14)
    # central differences on a few entries of every parameter
    h = 1e-6
    for pi, p in enumerate(net.params()):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, 4, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(net, zn, tn)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(net, zn, tn)
            flat[idx] = old
            assert (lp - lm) / (2 * h) == pytest.approx(g[pi].reshape(-1)[idx], rel=1e-5, abs=1e-10)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; the gradient passing back through it is rounded to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def test_bf16_backward_matches_autograd_with_the_same_rounding_points():
    """The BF16-emulating backward: every matrix-product operand rounded to bfloat16 -- the
    forward's inputs and weights (rounded values, gradient passed straight through) and the
    gradients entering the weight and input products (dy, dz2, dz1) -- while the bias
    gradients sum the unrounded ones.  Torch autograd with the roundings placed at those
    points by hand computes the same loss and gradients to 1e-12."""
    net = _net(7)
    rng = np.random.default_rng(4)
    zn, tn = rng.standard_normal((48, 16)), rng.standard_normal((48, 12))
    loss, g = mlp.loss_and_grads(net, zn, tn, bf16=True)

    t = lambda a: torch.tensor(a, dtype=torch.float64)
    rnd = lambda a: a.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    st = lambda a: a + (rnd(a) - a).detach()                     # rounded value, identity gradient
    W1, b1, W2, b2, W3, b3 = (t(p).requires_grad_(True) for p in net.params())
    a0 = st(t(zn))
    z1 = _RoundGrad.apply(a0 @ st(W1).T) + b1
    a1 = st(torch.tanh(z1))
    z2 = _RoundGrad.apply(a1 @ st(W2).T) + b2
    a2 = st(torch.tanh(z2))
    y = _RoundGrad.apply(a2 @ st(W3).T) + b3
    lt = torch.mean((y - t(tn)) ** 2)
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-13)
    for gi, p in zip(g, (W1, b1, W2, b2, W3, b3)):
        ref = p.grad.numpy()
        assert np.max(np.abs(gi - ref)) <= 1e-12 * max(1e-30, np.max(np.abs(ref)))
    # and the roundings matter: the FP64 backward differs from both by far more than that
    _, g64 = mlp.loss_and_grads(net, zn, tn, bf16=False)
    assert max(np.max(np.abs(a - b)) / np.max(np.abs(b)) for a, b in zip(g64, g)) > 1e-4


def test_adam_matches_torch():
    net = _net()
    rng = np.random.default_rng(3)
    ref = [torch.tensor(p.copy(), requires_grad=True) for p in net.params()]
    opt_t = torch.optim.Adam(ref, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    opt = mlp.Adam(net, lr=1e-3)
    for _ in range(5):
        grads = [rng.standard_normal(p.shape) for p in net.params()]
        opt.step(net, grads)
        for r, gr in zip(ref, grads):
            r.grad = torch.tensor(gr)
        opt_t.step()
    for p, r in zip(net.params(), ref):
        assert np.allclose(p, r.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_targets_are_one_euler_step():
    wl = W.quadrotor()
    x, u = W.mlp_training_inputs(100)
    from oracle import systems
    d = mlp.transitions(wl, x, u)
    assert np.allclose(d, wl.dt * systems.Quadrotor(wl.params).xdot(x, u), rtol=1e-13, atol=1e-16)


def test_training_reduces_the_loss():
    wl = W.quadrotor()
    x, u = W.mlp_training_inputs(20000)
    d = mlp.transitions(wl, x, u)
    z = np.concatenate([x, u], 1)
    mi, si, mo, so = mlp.standardisation(z, d)
    w = W.mlp_init_weights()
    net = mlp.Net(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"], mi, si, mo, so)
    zn, tn = (z - mi) / si, (d - mo) / so
    l0, _ = mlp.loss_and_grads(net, zn, tn)
    opt = mlp.Adam(net, lr=2e-3)
    for ep, order in enumerate(W.minibatch_order(20000, 3)):
        for s in range(0, 20000, 1000):
            _, g = mlp.loss_and_grads(net, zn[order[s:s + 1000]], tn[order[s:s + 1000]], bf16=True)
            opt.step(net, g)
    l1, _ = mlp.loss_and_grads(net, zn, tn)
    assert l1 < 0.25 * l0


def test_learned_step_replaces_euler():
    net = _net()
    wl = W.quadrotor()
    sysm = mlp.QuadrotorMLP(wl.params, net, bf16=False)
    x, u = W.mlp_training_inputs(10)
    from oracle import systems
    assert np.allclose(systems.euler_step(sysm, x, u, wl.dt), x + mlp.predict_delta(net, x, u), rtol=1e-14)


# ------------------------------------------------- element-wise bars of the GPU tests
from tests import _mlp_bounds as MB   # noqa: E402

F32 = np.float32


def _tanh_f32(x):
    e = np.exp(F32(2.0) * np.abs(x), dtype=F32)
    return np.copysign(F32(1.0) - F32(2.0) / (e + F32(1.0)), x).astype(F32)


def _fp32_network(net, zn, tn, mistake=None):
    """An FP32 realisation of the network's forward and backward with bfloat16 operands (what
    the GPU kernels compute, written independently with NumPy float32 products and sums):
    returns the standardised outputs and the six gradients.  `mistake` plants one error."""
    b16 = lambda a: MB.omlp.bf16_round(a).astype(F32)
    W1, W2, W3 = b16(net.W1), b16(net.W2), b16(net.W3)
    if mistake == "transposed_W2":
        W2 = W2.T.copy()
    b1, b2, b3 = (np.asarray(b, dtype=F32) for b in (net.b1, net.b2, net.b3))
    if mistake == "dropped_b2":
        b2 = np.zeros_like(b2)
    a0 = b16(zn)
    h1 = _tanh_f32(a0 @ W1.T + b1)
    a1 = b16(h1)
    h2 = _tanh_f32(a1 @ W2.T + b2)
    a2 = b16(h2)
    y = a2 @ W3.T + b3
    B = zn.shape[0]
    g = ((F32(1.0) if mistake == "loss_gradient_without_2" else F32(2.0)) * (y - tn.astype(F32))
         / F32(B * 12)).astype(F32)
    gr = b16(g)
    s2 = F32(1.0) + h2 * h2 if mistake == "tanh_derivative_sign" else F32(1.0) - h2 * h2
    dz2 = (gr @ W3) * s2
    dz2r = b16(dz2)
    dz1 = (dz2r @ W2) * (F32(1.0) - h1 * h1)
    dz1r = b16(dz1)
    col = lambda v: v.astype(np.float64).sum(axis=0).astype(F32)
    gW2 = dz2r.T @ (a2 if mistake == "wrong_layer_in_weight_gradient" else a1)
    grads = [dz1r.T @ a0, col(dz1), gW2, col(dz2), gr.T @ a2, col(g)]
    return y.astype(np.float64), [np.asarray(x, dtype=np.float64) for x in grads]


def _bounds_case(n=4096):
    wl = W.quadrotor()
    x, u = W.mlp_training_inputs(n)
    d = mlp.transitions(wl, x, u)
    z = np.concatenate([x, u], 1)
    mi, si, mo, so = mlp.standardisation(z, d)
    w = W.mlp_init_weights(5)
    rng = np.random.default_rng(1)
    net = mlp.Net(w["W1"], w["b1"] + 0.1 * rng.standard_normal(128), w["W2"], w["b2"] + 0.1 * rng.standard_normal(128),
                  w["W3"], w["b3"] + 0.1 * rng.standard_normal(12), mi, si, mo, so)
    return net, (z - mi) / si, (d - mo) / so


def _worst(got, ref, bound):
    return float(np.max(np.abs(got - ref) / bound))


@pytest.mark.parametrize("n", [48, 4096])
def test_elementwise_bounds_hold_for_an_fp32_realisation(n):
    """The per-element bounds of the GPU MLP tests (tests/_mlp_bounds.py) hold for an
    independent FP32 realisation of the same bfloat16 arithmetic, on every output of the
    forward and every element of every gradient, including the elements whose bfloat16
    operands flip between FP32 and FP64 (a small batch and a full minibatch)."""
    net, zn, tn = _bounds_case(n)
    y_ref, _ = mlp.forward_normalised(net, zn, bf16=True)
    _, g_ref = mlp.loss_and_grads(net, zn, tn, bf16=True)
    y32, g32 = _fp32_network(net, zn, tn)
    yb, _ = MB.forward_bounds(net, zn)
    assert np.any(y32 != y_ref)                         # the realisations differ ...
    assert _worst(y32, y_ref, yb) <= 1.0                # ... within the bound
    for k, (a, b, bd) in enumerate(zip(g32, g_ref, MB.gradient_bounds(net, zn, tn))):
        assert _worst(a, b, bd) <= 1.0, (k, _worst(a, b, bd))


@pytest.mark.parametrize("mistake", ["dropped_b2", "transposed_W2", "tanh_derivative_sign",
                                     "loss_gradient_without_2", "wrong_layer_in_weight_gradient"])
@pytest.mark.parametrize("n", [48, 4096])
def test_elementwise_bounds_catch_planted_mistakes(mistake, n):
    """Each planted mistake in the FP32 realisation (a dropped term, a transposed operand, a
    wrong sign, factor or operand) breaks the bound on some element by far.  A mistake of one
    bfloat16 step (a rounding placed at another point) stays inside the flip allowance; the
    oracle's own rounding points are pinned against torch autograd above."""
    net, zn, tn = _bounds_case(n)
    y_ref, _ = mlp.forward_normalised(net, zn, bf16=True)
    _, g_ref = mlp.loss_and_grads(net, zn, tn, bf16=True)
    y32, g32 = _fp32_network(net, zn, tn, mistake=mistake)
    yb, _ = MB.forward_bounds(net, zn)
    worst = max([_worst(y32, y_ref, yb)] + [_worst(a, b, bd) for a, b, bd in
                                           zip(g32, g_ref, MB.gradient_bounds(net, zn, tn))])
    assert worst > 10.0, worst
