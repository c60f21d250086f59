"""The allocation-free control step (mppi_step_static) through the C ABI: two calls in a row on
one GPU, the second with a smaller problem, each bit for bit what the context path
(mppi_create, the state restored to the same sequence and noise counter, mppi_step) computes,
and the second also against the FP64 oracle."""
import struct

import numpy as np
import pytest

import paper_1509_01149_amd as P
import workloads as W
from oracle import mppi
from tests._parity import TOL_U

pytestmark = pytest.mark.gpu


def _context_step(wl, x0, U, iteration, n_iters):
    with P.controller_for(wl) as c:
        c.set_state(struct.pack("<QQQ", 0x4d50504953544131, U.size, iteration) + U.astype("<f8").tobytes())
        u0 = c.step(x0, n_iters)
        return u0, c.get_controls(), c.iteration()


def _start(wl, seed):
    rng = np.random.default_rng(seed)
    U = mppi.initial_sequence(wl) + 0.1 * rng.standard_normal((wl.T, wl.m))
    return U, (1 << 33) + 17 * seed


SEQUENCES = {
    "bicycle_then_smaller_bicycle": [lambda: W.bicycle(K=8192, T=100), lambda: W.bicycle(K=1000, T=37)],
    "quadrotor_then_cartpole": [lambda: W.quadrotor(nu=2.0, K=16384, T=150), lambda: W.cartpole(nu=2.0, K=999, T=60)],
}


@pytest.mark.parametrize("name", list(SEQUENCES))
def test_static_step_equals_context_step(name):
    for call, make in enumerate(SEQUENCES[name]):
        wl = make().replace(seed=40 + call)
        U, it = _start(wl, call + 1)
        n_iters = 2 if call == 0 else 1
        print(name, "call", call, wl.name, "K", wl.K, "T", wl.T, flush=True)
        u0_s, U_s, it_s = P.step_static(wl.x0, U, it, n_iters, **P.controller_args(wl))
        u0_c, U_c, it_c = _context_step(wl, wl.x0, U, it, n_iters)
        assert it_s == it_c == it + n_iters
        assert np.array_equal(u0_s, u0_c) and np.array_equal(U_s, U_c)
        if call == 1:       # the smaller problem also against the oracle
            u0_r, U_r, it_r, _ = mppi.control_step(wl, wl.x0, U, it)
            scale = max(1.0, float(np.max(np.abs(U_r))))
            assert it_r == it_s
            assert max(np.max(np.abs(u0_s - u0_r)), np.max(np.abs(U_s - U_r))) / scale <= TOL_U


def test_static_step_rejects_what_does_not_fit():
    wl = W.bicycle(K=1 << 20, T=100)
    U, it = _start(wl, 3)
    with pytest.raises(P.MppiError) as e:
        P.step_static(wl.x0, U, it, 1, **P.controller_args(wl))
    assert e.value.code == P.binding.EINVAL and "static scratch" in str(e.value)
