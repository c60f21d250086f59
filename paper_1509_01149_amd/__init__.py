"""MI355X-native MPPI with covariance-variable importance sampling (arXiv 1509.01149).

The hot path (noise, rollouts, likelihood-ratio costs, weights, FP64 update, warm
shift) runs in the HIP kernels of libmppi.so behind the C ABI in include/mppi.h;
``binding`` is a thin ctypes layer over it.
"""
from .binding import (  # noqa: F401
    ABI_VERSION, Controller, Mlp, MppiError, NumericError, Server, load, philox, step_static, version,
    SERVE_BATCHED, SERVE_PLAIN, SERVE_BATCHED_GRAPH, WEIGHT_PATH, WEIGHT_COST_TO_GO,
    KERNELS_AUTO, KERNELS_FUSED, KERNELS_THREE,
    SYS_LINEAR, SYS_CARTPOLE, SYS_BICYCLE, SYS_QUADROTOR, SYS_QUADROTOR_MLP, SYS_CARTPOLE_SWINGUP,
)


def controller_args(wl, **kw) -> dict:
    """Keyword arguments of Controller / Server.admit from any object with the fields of a
    workload description (system, n, m, K, T, dt, lam, nu, sigma, R, u_init, params, seed)."""
    args = dict(system=wl.system, n=wl.n, m=wl.m, K=wl.K, T=wl.T, dt=wl.dt, lam=wl.lam, nu=wl.nu,
                sigma=wl.sigma, R=wl.R, u_init=wl.u_init, params=wl.params, seed=wl.seed)
    args.update(kw)
    return args


def controller_for(wl, **kw) -> Controller:
    return Controller(**controller_args(wl, **kw))
