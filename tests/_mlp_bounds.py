"""Element-wise error bounds of the BF16 network (FP32 accumulation, bfloat16 operands) against
the FP64 oracle that rounds the same operands to bfloat16, derived from the arithmetic.

Both sides round every matrix-product operand to bfloat16.  Where the FP64 value of an
operand lies so close to a bfloat16 rounding boundary that the FP32 computation can fall on
the other side, the two sides hold different operands (a "flip": one bfloat16 step); every
other operand is the same bfloat16 number on both sides.  The bound of each element is then
  (a) the worst-case FP32 summation error of its own product or sum (any order, any tree):
      2 n 2^-24 sum |terms| for n terms (a factor 2 for the matrix cores' internal rounding),
      plus one rounding of the bias and of the result, and
  (b) the propagation of every operand that can flip or shift, through the absolute values
      of the downstream weights and tanh derivatives (first order; the margins below cover
      the second-order remainder).
An operand can flip when the interval [v - w, v + w] around its FP64 value v contains a
rounding boundary, w being the bound on its FP32 value's error; its bfloat16 value can then
be any of those the interval rounds to.  tanh is evaluated in FP32 from the hardware
exponential and reciprocal; its error is taken as 2^-21 absolute (the construction
1 - 2 / (e + 1) loses at most a few FP32 ulps of 1).

The bounds hold for any correct FP32 realisation of the same products; a mistake that changes
a term (a dropped bias, a transposed weight, a wrong row) moves elements by O(1) relative and
fails them.  tests/test_oracle_mlp.py checks both statements on the CPU with a float32
emulation.
"""
import numpy as np

from oracle import mlp as omlp

U32 = 2.0 ** -24
TANH_ERR = 2.0 ** -21
MARGIN = 1.01


def _spread(v, w):
    """Largest difference between the bfloat16 roundings of any two points of [v - w, v + w]
    (0 where the whole interval rounds to one value)."""
    return np.abs(omlp.bf16_round(v + w) - omlp.bf16_round(v - w))


def _acc(n, absterms):
    return 2.0 * n * U32 * absterms


def forward_bounds(net, zn):
    """Per-element bound on |y_gpu - y_orc| for standardised outputs y (B, 12), with the
    intermediate quantities the backward bounds need."""
    a0 = omlp.bf16_round(zn)
    W1, W2, W3 = (omlp.bf16_round(net.W1), omlp.bf16_round(net.W2), omlp.bf16_round(net.W3))
    b1, b2, b3 = net.b1, net.b2, net.b3
    z1 = a0 @ W1.T + b1
    h1 = np.tanh(z1)
    # layer 1: 16 products; the bias is the FP32 copy of the FP64 value (one rounding) and the
    # bias add rounds once; a0 is the same on both sides (standardisation in FP64 first)
    e1 = _acc(16, np.abs(a0) @ np.abs(W1).T) + U32 * np.abs(b1) + U32 * np.abs(z1)
    dh1 = MARGIN * (1.0 - h1 * h1) * e1 + TANH_ERR           # |h1_gpu - h1| (FP32, unrounded)
    da1 = _spread(h1, dh1)                                   # |a1_gpu - a1|
    a1 = omlp.bf16_round(h1)
    z2 = a1 @ W2.T + b2
    h2 = np.tanh(z2)
    e2 = _acc(128, np.abs(a1) @ np.abs(W2).T) + U32 * np.abs(b2) + U32 * np.abs(z2) + da1 @ np.abs(W2).T
    dh2 = MARGIN * (1.0 - h2 * h2) * e2 + TANH_ERR
    da2 = _spread(h2, dh2)
    a2 = omlp.bf16_round(h2)
    y = a2 @ W3.T + b3
    dy = (_acc(128, np.abs(a2) @ np.abs(W3).T) + U32 * np.abs(b3) + U32 * np.abs(y)
          + MARGIN * (da2 @ np.abs(W3).T) + 1e-12 * (1.0 + np.abs(y)))
    return dy, dict(a0=a0, a1=a1, a2=a2, h1=h1, h2=h2, dh1=dh1, dh2=dh2, da1=da1, da2=da2, y=y, dy=dy,
                    W1=W1, W2=W2, W3=W3)


def gradient_bounds(net, zn, tn):
    """Per-element bounds on the six gradients [gW1, gb1, gW2, gb2, gW3, gb3] of the mean
    squared error (the oracle's loss_and_grads with bf16=True), as the GPU's kernels form
    them: dY = 2 (Y - T) / (12 B) in FP32 (T rounded to FP32), bfloat16 copies of dY, dZ2 and
    dZ1 for the products, FP32 copies for the bias gradients (column sums in FP64)."""
    B = zn.shape[0]
    c = 2.0 / (B * omlp.N_OUT)
    dyb, f = forward_bounds(net, zn)
    a0, a1, a2, h1, h2 = f["a0"], f["a1"], f["a2"], f["h1"], f["h2"]
    W2, W3 = f["W2"], f["W3"]
    diff = f["y"] - tn
    g = c * diff
    # |dY_gpu - dY|: the output's bound, T's FP32 rounding, three FP32 roundings of the result
    dg = c * (dyb + U32 * np.abs(tn)) + 3.0 * U32 * np.abs(g)
    dgr = _spread(g, dg)
    gr = omlp.bf16_round(g)
    # dZ2 = (dYr W3) (1 - H2^2): 12 products, then FP32 products with the FP32 tanh
    p2 = gr @ W3
    dp2 = _acc(12, np.abs(gr) @ np.abs(W3)) + dgr @ np.abs(W3)
    s2 = 1.0 - h2 * h2
    ds2 = MARGIN * 2.0 * np.abs(h2) * f["dh2"] + 2.0 * U32
    dz2 = p2 * s2
    ddz2 = MARGIN * (dp2 * s2 + np.abs(p2) * ds2 + dp2 * ds2) + U32 * np.abs(dz2)
    ddz2r = _spread(dz2, ddz2)
    dz2r = omlp.bf16_round(dz2)
    # dZ1 = (dZ2r W2) (1 - H1^2): 128 products
    p1 = dz2r @ W2
    dp1 = _acc(128, np.abs(dz2r) @ np.abs(W2)) + ddz2r @ np.abs(W2)
    s1 = 1.0 - h1 * h1
    ds1 = MARGIN * 2.0 * np.abs(h1) * f["dh1"] + 2.0 * U32
    dz1 = p1 * s1
    ddz1 = MARGIN * (dp1 * s1 + np.abs(p1) * ds1 + dp1 * ds1) + U32 * np.abs(dz1)
    ddz1r = _spread(dz1, ddz1)
    dz1r = omlp.bf16_round(dz1)

    def wgrad(d, dd, a, da):
        # sum over the batch of d^T a with operands off by dd and da (B terms, FP32 result)
        val = d.T @ a
        return (_acc(B, np.abs(d).T @ np.abs(a)) + MARGIN * (dd.T @ np.abs(a) + np.abs(d).T @ da + dd.T @ da)
                + U32 * np.abs(val))

    def bgrad(v, dv):
        # FP64 column sum of FP32 values, rounded to FP32 once
        s = v.sum(axis=0)
        return dv.sum(axis=0) + _acc(B, np.abs(v).sum(axis=0)) * 2.0 ** -29 + U32 * np.abs(s)

    zero_a0 = np.zeros_like(a0)
    return [wgrad(dz1r, ddz1r, a0, zero_a0), bgrad(dz1, ddz1),
            wgrad(dz2r, ddz2r, a1, f["da1"]), bgrad(dz2, ddz2),
            wgrad(gr, dgr, a2, f["da2"]), bgrad(g, dg)]
