"""The two-kernel iteration (rollout blocks that keep their normals in LDS and also form their
samples' weighted noise sums against their own minimum; a multi-block finalize that rescales
and merges them) against the three-kernel iteration (rollout, update, finalize) on the same
inputs, through the C ABI: the step-split systems and the quadrotor's four-lane body.

Both compute the update law of Section III-C from the same path costs and the same normals;
the per-block factor exp(-(rho_b - rho)/lambda) is the sample-independent factor that
cancels in the normalised update (Section III-B), so the two differ by FP64 summation order
only: costs and minima bitwise, the normaliser and the update within a bound of FP64
reassociation over K terms.
"""
import numpy as np
import pytest
import torch

import paper_1509_01149_amd as P
import workloads as W
from oracle import mppi
from tests._parity import assert_parity, one_step

pytestmark = pytest.mark.gpu

# FP64 sums of up to 16384 terms in two orders: |difference| <= 2 K 2^-53 sum |terms|; the
# weighted noise sums cancel (sum |w eps| / |sum w eps| grows like sqrt of the effective
# sample count), so the bar is taken relative to the largest component, with that headroom
TOL_ETA = 1e-12
TOL_DU = 1e-9
# later iterations: the two FP64 masters may round to different FP32 copies (one ulp apart)
# for the next rollout, after which the costs differ in their last FP32 bits
TOL_LATER = 1e-6

CASES = [
    W.bicycle(),                                                       # 32 lanes, 512 blocks
    W.bicycle(K=8192, T=40),                                           # 16 lanes, 512 blocks
    W.bicycle(K=1000, T=37),                                           # ragged K and T*m
    W.bicycle(K=2048, T=60).replace(sigma=np.array([[0.5, 0.1], [0.1, 0.3]])),   # full covariance
    W.bicycle(K=1024, T=30, nu=np.array([1.0, 4.0])),                  # per-dimension nu
    W.bicycle(K=4096, T=512),                                          # normals at the 32 KiB LDS limit
    W.cartpole(nu=2.0),
    W.cartpole(K=257, T=7),                                            # one finalize block
    W.cartpole(K=65536, T=16),                                         # 4 lanes, 1024 blocks
    W.cartpole_swingup(nu=100.0),
    W.linear_double_integrator(K=300, R=0.3),
    W.quadrotor(),                                                     # 256 blocks, 150 KiB of normals each
    W.quadrotor(K=1000, T=37),                                         # ragged K
    W.quadrotor(K=2048, T=153),                                        # the longest horizon whose normals fit
    W.quadrotor(K=2048, T=80).replace(sigma=0.2 * np.eye(4) + 0.05 * np.ones((4, 4))),   # full covariance
    W.quadrotor(nu=np.array([1.0, 2.0, 4.0, 8.0]), lam=420.0, K=4096, T=60),              # per-dimension nu
    W.quadrotor(K=4096, T=150, crash=True),                            # the crash indicator
    W.quadrotor(K=2048, T=100, obstacles=W.obstacle_field(n=100)),     # 68 obstacles read from LDS
    W.quadrotor(K=2048, T=100, obstacles=W.obstacle_field(n=100), crash=True),
]


def _ids(wl):
    return f"{wl.name}-K{wl.K}-T{wl.T}"


def _pair(wl):
    return (P.controller_for(wl, kernels=P.KERNELS_FUSED), P.controller_for(wl, kernels=P.KERNELS_THREE))


@pytest.mark.parametrize("wl", CASES, ids=_ids)
def test_fused_iteration_equals_three_kernel_iteration(wl):
    f, t = _pair(wl)
    with f, t:
        fi, ti = f.info(), t.info()
        assert fi["rollout_mode"] & P.binding.ROLLOUT_FUSED and fi["update_blocks"] == 0, fi
        assert not ti["rollout_mode"] & P.binding.ROLLOUT_FUSED and ti["update_blocks"] > 0, ti
        uf, ut = f.step(wl.x0), t.step(wl.x0)
        Sf, rf, ef, dUf = f.debug_last()
        St, rt, et, dUt = t.debug_last()
        assert np.array_equal(Sf, St)                         # the same rollouts
        assert rf == rt
        assert abs(ef - et) <= TOL_ETA * et, (ef, et)
        scale = float(np.max(np.abs(dUt)))
        assert np.max(np.abs(dUf - dUt)) <= TOL_DU * scale, (np.max(np.abs(dUf - dUt)), scale)
        Uf, Ut = f.get_controls(), t.get_controls()
        U_scale = max(1.0, float(np.max(np.abs(Ut))))
        assert np.max(np.abs(Uf - Ut)) <= TOL_DU * U_scale
        assert np.max(np.abs(uf - ut)) <= TOL_DU * U_scale
        for it in (1, 2):
            uf, ut = f.step(wl.x0), t.step(wl.x0)
            Uf, Ut = f.get_controls(), t.get_controls()
            U_scale = max(1.0, float(np.max(np.abs(Ut))))
            assert np.max(np.abs(Uf - Ut)) <= TOL_LATER * U_scale, it
            assert np.max(np.abs(uf - ut)) <= TOL_LATER * U_scale, it
        assert f.iteration() == t.iteration() == 3


@pytest.mark.parametrize("kernels", [P.KERNELS_FUSED, P.KERNELS_THREE], ids=["fused", "three"])
def test_both_iterations_match_the_oracle(kernels):
    """First iteration at full size against the FP64 oracle, to the parity bars (the library
    picks the fused iteration for these by default; the three-kernel one is asked for)."""
    for wl in (W.bicycle().replace(seed=5), W.cartpole(nu=2.0).replace(seed=5),
               W.cartpole_swingup(nu=100.0).replace(seed=5), W.quadrotor(K=2048).replace(seed=5)):
        with P.controller_for(wl, kernels=kernels) as c:
            fused = bool(c.info()["rollout_mode"] & P.binding.ROLLOUT_FUSED)
            assert fused == (kernels == P.KERNELS_FUSED)
            m = one_step(wl, c, wl.x0, mppi.initial_sequence(wl), 0)
        assert_parity(m, label=f"{wl.name} kernels={kernels}")


CTG_CASES = [
    W.bicycle(),                                                       # 32 lanes, 512 blocks
    W.bicycle(K=1000, T=37),                                           # ragged K and T*m
    W.bicycle(K=2048, T=60).replace(sigma=np.array([[0.5, 0.1], [0.1, 0.3]])),   # full covariance
    W.cartpole(nu=2.0),                                                # m = 1: four steps per finalize block
    W.cartpole(K=257, T=7),                                            # one finalize block, ragged
    W.linear_double_integrator(K=300, R=0.3),
]


@pytest.mark.parametrize("wl", CTG_CASES, ids=_ids)
def test_fused_cost_to_go_equals_three_kernel_cost_to_go(wl):
    """Cost-to-go weighting through two kernels (each rollout block weights its samples'
    steps against its own per-step minima, the finalize rescales by
    exp(-(rho_b,i - rho_i)/lambda) per step) against the three-kernel iteration: the same
    costs bitwise, each step's minimum exactly, the normaliser and the update to FP64
    reassociation."""
    ctg = P.WEIGHT_COST_TO_GO
    f = P.controller_for(wl, weighting=ctg, kernels=P.KERNELS_FUSED)
    t = P.controller_for(wl, weighting=ctg, kernels=P.KERNELS_THREE)
    with f, t:
        fi, ti = f.info(), t.info()
        assert fi["rollout_mode"] & P.binding.ROLLOUT_FUSED and fi["update_blocks"] == 0, fi
        assert not ti["rollout_mode"] & P.binding.ROLLOUT_FUSED, ti
        uf, ut = f.step(wl.x0), t.step(wl.x0)
        Sf, rf, ef, dUf = f.debug_last()
        St, rt, et, dUt = t.debug_last()
        assert np.array_equal(Sf, St)
        assert rf == rt                                 # step 0's minimum (the path minimum)
        assert abs(ef - et) <= TOL_ETA * et, (ef, et)   # step 0's normaliser
        scale = float(np.max(np.abs(dUt)))
        assert np.max(np.abs(dUf - dUt)) <= TOL_DU * scale, (np.max(np.abs(dUf - dUt)), scale)
        U_scale = max(1.0, float(np.max(np.abs(t.get_controls()))))
        assert np.max(np.abs(f.get_controls() - t.get_controls())) <= TOL_DU * U_scale
        assert np.max(np.abs(uf - ut)) <= TOL_DU * U_scale
        for it in (1, 2):
            uf, ut = f.step(wl.x0), t.step(wl.x0)
            U_scale = max(1.0, float(np.max(np.abs(t.get_controls()))))
            assert np.max(np.abs(f.get_controls() - t.get_controls())) <= TOL_LATER * U_scale, it
        assert f.iteration() == t.iteration() == 3


def test_fused_closed_loop_with_the_plant():
    """The fused finalize with the plant step: a closed-loop run equals single steps bitwise,
    and stays with the three-kernel run to FP64 reassociation."""
    dev = torch.device("cuda:0")
    for wl in (W.bicycle(K=2048, T=50), W.cartpole(nu=2.0), W.cartpole_swingup(nu=1000.0, K=1024, T=50),
               W.quadrotor(K=2048, T=100)):
        wl = wl.replace(seed=41)
        n = 7
        xs = {k: torch.tensor(wl.x0, dtype=torch.float64, device=dev) for k in ("run", "single", "three")}
        logs = {k: torch.zeros((n, wl.m), dtype=torch.float64, device=dev) for k in xs}
        with P.controller_for(wl) as a, P.controller_for(wl) as b, \
                P.controller_for(wl, kernels=P.KERNELS_THREE) as c:
            assert a.info()["rollout_mode"] & P.binding.ROLLOUT_FUSED
            a.run_closed_loop_async(xs["run"].data_ptr(), n, logs["run"].data_ptr())
            for j in range(n):
                b.step_plant_async(xs["single"].data_ptr(), logs["single"][j].data_ptr())
            c.run_closed_loop_async(xs["three"].data_ptr(), n, logs["three"].data_ptr())
            a.sync(), b.sync(), c.sync()
            assert torch.equal(xs["run"], xs["single"]) and torch.equal(logs["run"], logs["single"])
            scale = max(1.0, float(logs["three"].abs().max()))
            assert float((logs["run"] - logs["three"]).abs().max()) <= TOL_LATER * scale, wl.name
            assert float((xs["run"] - xs["three"]).abs().max()) <= TOL_LATER * max(1.0, float(xs["three"].abs().max()))
            assert a.iteration() == c.iteration() == n
