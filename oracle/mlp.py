"""Learned dynamics surrogate, FP64 (test infrastructure only).

An MLP [16 -> 128 -> 128 -> 12] with tanh hidden layers maps the standardised
(state, control) of the quadrotor to its standardised one-step state change; the
rollout then steps x <- x + dx.  The paper's method needs only a dynamics model to
sample from (Section II, Algorithm 1), so a learned model slots in where f, G were.

``bf16=True`` emulates the GPU's arithmetic: every matrix-product input (weights and
activations, forward and backward) is rounded to bfloat16 (round to nearest even,
through FP32 as the GPU holds it); products and sums are then exact in FP64, where the
GPU accumulates in FP32.

Loss: mean squared error over the batch and the 12 outputs of the standardised
target.  Optimiser: Adam (Kingma & Ba, 2015) on FP32 master weights.
"""
import numpy as np

from . import systems as _systems

H = 128
N_IN = 16
N_OUT = 12


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), via FP32; returns float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(a, bf16):
    return bf16_round(a) if bf16 else np.asarray(a, dtype=np.float64)


class Net:
    """Weights W1 (128, 16), W2 (128, 128), W3 (12, 128), biases, and standardisation
    statistics of inputs (mu_in, sd_in: 16) and targets (mu_out, sd_out: 12)."""

    def __init__(self, W1, b1, W2, b2, W3, b3, mu_in, sd_in, mu_out, sd_out):
        self.W1, self.b1, self.W2, self.b2, self.W3, self.b3 = (np.array(a, dtype=np.float64)
                                                                for a in (W1, b1, W2, b2, W3, b3))
        self.mu_in, self.sd_in = np.array(mu_in, float), np.array(sd_in, float)
        self.mu_out, self.sd_out = np.array(mu_out, float), np.array(sd_out, float)

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]

    def copy(self):
        return Net(*self.params(), self.mu_in, self.sd_in, self.mu_out, self.sd_out)


def forward_normalised(net, zn, bf16=False):
    """Standardised input zn (B, 16) -> standardised output y (B, 12) and the cache."""
    a0 = _r(zn, bf16)
    z1 = a0 @ _r(net.W1, bf16).T + net.b1
    h1 = np.tanh(z1)
    a1 = _r(h1, bf16)
    z2 = a1 @ _r(net.W2, bf16).T + net.b2
    h2 = np.tanh(z2)
    a2 = _r(h2, bf16)
    y = a2 @ _r(net.W3, bf16).T + net.b3
    return y, (a0, h1, a1, h2, a2)


def predict_delta(net, x, u, bf16=False):
    """One-step state change dx for states x (B, 12) and controls u (B, 4)."""
    z = np.concatenate([x, u], axis=1)
    y, _ = forward_normalised(net, (z - net.mu_in) / net.sd_in, bf16)
    return y * net.sd_out + net.mu_out


def loss_and_grads(net, zn, tn, bf16=False):
    """MSE of the standardised prediction and its exact gradients (chain rule)."""
    B = zn.shape[0]
    y, (a0, h1, a1, h2, a2) = forward_normalised(net, zn, bf16)
    diff = y - tn
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / (B * N_OUT)
    dyr = _r(dy, bf16)
    gW3 = dyr.T @ a2
    gb3 = dy.sum(axis=0)
    dz2 = (dyr @ _r(net.W3, bf16)) * (1.0 - h2 * h2)
    dz2r = _r(dz2, bf16)
    gW2 = dz2r.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2r @ _r(net.W2, bf16)) * (1.0 - h1 * h1)
    gW1 = _r(dz1, bf16).T @ a0
    gb1 = dz1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


class Adam:
    def __init__(self, net, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros_like(p) for p in net.params()]
        self.v = [np.zeros_like(p) for p in net.params()]
        self.t = 0

    def step(self, net, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(net.params(), grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def transitions(workload, x, u):
    """Targets: the analytic one-step change dx = dt f(x, u) of the quadrotor (one Euler step)."""
    quad = _systems.Quadrotor(workload.params)
    return workload.dt * quad.xdot(x, u)


def standardisation(z, d):
    return z.mean(axis=0), z.std(axis=0), d.mean(axis=0), d.std(axis=0)


class QuadrotorMLP(_systems.Quadrotor):
    """The quadrotor's costs with the learned one-step model: x <- x + MLP(x, u)."""

    def __init__(self, params, net, bf16=True):
        super().__init__(params)
        self.net = net
        self.bf16 = bf16

    def step(self, x, v, dt):
        return x + predict_delta(self.net, x, v, self.bf16)
