"""Controller state through the C ABI on the GPU: the warm start of Algorithm 1 (the nominal
sequence U and the iteration counter that keys the noise) is the whole controller state, so
a snapshot restored into a fresh context continues bit for bit; a sequence set from the host
is the one the next iteration starts from; a workspace lent by torch gives the same results
as the library's own allocation."""
import numpy as np
import pytest

import paper_1509_01149_amd as P
import workloads as W
from oracle import mppi
from tests._parity import assert_parity, controller, one_step

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("make", [lambda: W.cartpole(nu=2.0, K=1000, T=100),
                                  lambda: W.quadrotor(nu=2.0, K=2048, T=60),
                                  lambda: W.bicycle(K=4096, T=100)])
def test_snapshot_restore_continues_bitwise(make):
    """Run 40 closed-loop steps, snapshot, run 40 more; restore the snapshot into a fresh
    context and run the same 40: identical controls, sequences and iteration counters."""
    wl = make().replace(seed=41)
    x = wl.x0.copy()
    with controller(wl) as a:
        for _ in range(40):
            x = mppi.plant_step(wl, x, a.step(x))
        blob, x_snap = a.get_state(), x.copy()
        it_snap = a.iteration()
        ua = []
        for _ in range(40):
            u = a.step(x)
            ua.append(u)
            x = mppi.plant_step(wl, x, u)
        Ua, ita = a.get_controls(), a.iteration()
    with controller(wl) as b:
        b.set_state(blob)
        assert b.iteration() == it_snap == 40
        x = x_snap
        ub = []
        for _ in range(40):
            u = b.step(x)
            ub.append(u)
            x = mppi.plant_step(wl, x, u)
        assert np.array_equal(np.array(ua), np.array(ub))
        assert np.array_equal(b.get_controls(), Ua) and b.iteration() == ita == 80


def test_snapshot_rejects_a_mismatched_context():
    wl = W.cartpole(K=256, T=50).replace(seed=42)
    with controller(wl) as a, controller(wl.replace(T=40)) as b:
        blob = a.get_state()
        with pytest.raises(P.MppiError) as e:
            b.set_state(blob)
        assert e.value.code == P.binding.EINVAL
        with pytest.raises(P.MppiError):
            a.set_state(blob[:-8])                         # truncated


def test_set_controls_is_the_next_iterations_start():
    """A sequence set from the host (and an iteration counter from a snapshot) is exactly what
    the next iteration starts from: parity with the oracle from that sequence and iteration."""
    wl = W.quadrotor(nu=2.0, K=4096, T=100).replace(seed=43)
    rng = np.random.default_rng(0)
    U = mppi.initial_sequence(wl) + 0.3 * rng.standard_normal((wl.T, wl.m))
    with controller(wl) as c:
        c.set_controls(U)
        assert np.array_equal(c.get_controls(), U)
        blob = bytearray(c.get_state())
        blob[16:24] = int(7).to_bytes(8, "little")        # the iteration counter word
        c.set_state(bytes(blob))
        assert c.iteration() == 7 and np.array_equal(c.get_controls(), U)
        m = one_step(wl, c, wl.x0, U, 7)
    assert_parity(m, label="set_controls quadrotor")
    with pytest.raises(P.MppiError):
        with controller(wl) as c:
            c.set_controls(np.full((wl.T, wl.m), np.nan))


@pytest.mark.parametrize("make", [lambda: W.bicycle(K=4096, T=100), lambda: W.quadrotor(nu=2.0, K=4096, T=80)])
def test_torch_workspace_equals_library_allocation(make):
    import torch
    wl = make().replace(seed=44)
    stream = torch.cuda.Stream()
    with controller(wl) as a, controller(wl, torch_workspace=True, torch_stream=stream) as b:
        assert b._workspace is not None and b._workspace.numel() >= b.info()["workspace_bytes"]
        x = wl.x0.copy()
        for _ in range(5):
            ua, ub = a.step(x), b.step(x)
            assert np.array_equal(ua, ub)
            x = mppi.plant_step(wl, x, ua)
        assert np.array_equal(a.get_controls(), b.get_controls())
        Sa, ra, ea, dUa = a.debug_last()
        Sb, rb, eb, dUb = b.debug_last()
        assert np.array_equal(Sa, Sb) and ra == rb and ea == eb and np.array_equal(dUa, dUb)
