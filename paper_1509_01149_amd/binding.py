"""ctypes binding of libmppi (argument marshalling only).

Every step of the MPPI iteration runs in the HIP kernels behind the C ABI declared in
include/mppi.h; this module only converts Python/NumPy arguments into the ABI's
structs and pointers.  PyTorch is used, when asked, for device memory (a lent
workspace) and for the stream to run on.  There is no fallback: if libmppi.so is not
built, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MPPI_LIBRARY names another build of the same library (the sanitizer build of the host
# code); it must exist like the default one
LIB_PATH = os.environ.get("MPPI_LIBRARY") or os.path.join(_HERE, "libmppi.so")

ABI_VERSION = 1
OK, EINVAL, ENOMEM, EDEVICE, EBUSY, ENUMERIC, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
SYS_LINEAR, SYS_CARTPOLE, SYS_BICYCLE, SYS_QUADROTOR, SYS_QUADROTOR_MLP, SYS_CARTPOLE_SWINGUP = 0, 1, 2, 3, 4, 5

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_u32p = C.POINTER(C.c_uint32)
_u64p = C.POINTER(C.c_uint64)


class MppiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libmppi error {code}: {msg}")
        self.code = code


class NumericError(MppiError):
    """An iteration had no sample with a finite path cost (status MPPI_ENUMERIC)."""


class LinearParams(C.Structure):
    _fields_ = [("A", _dp), ("B", _dp), ("Q", _dp), ("Qf", _dp)]


class CartPoleParams(C.Structure):
    _fields_ = [("mass_cart", C.c_double), ("mass_pole", C.c_double), ("half_length", C.c_double),
                ("gravity", C.c_double), ("q_diag", C.c_double * 4), ("qf_diag", C.c_double * 4)]


class SwingUpParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("gain", "half_length", "gravity", "w_pos", "w_angle", "w_vel", "w_rate")]


class BicycleParams(C.Structure):
    _fields_ = [("wheelbase", C.c_double), ("v_target", C.c_double), ("w_speed", C.c_double),
                ("cell_size", C.c_double), ("steer_limit", C.c_double), ("map_w", C.c_int32),
                ("map_h", C.c_int32), ("map", _fp)]


class QuadrotorParams(C.Structure):
    _fields_ = [("mass", C.c_double), ("gravity", C.c_double), ("arm", C.c_double), ("yaw_coef", C.c_double),
                ("inertia", C.c_double * 3), ("goal", C.c_double * 3), ("w_goal", C.c_double),
                ("w_obs", C.c_double), ("obs_margin", C.c_double), ("n_obstacles", C.c_int32),
                ("obstacles", _dp), ("crash_cost", C.c_double), ("ground_z", C.c_double)]


class QuadrotorMlpParams(C.Structure):
    _fields_ = [("quad", QuadrotorParams), ("mlp", C.c_void_p)]


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("system", C.c_int32), ("n_state", C.c_int32), ("n_ctrl", C.c_int32),
                ("K", C.c_int32), ("T", C.c_int32), ("dt", C.c_double), ("lambda_", C.c_double),
                ("nu", C.c_double), ("sigma", _dp), ("R", _dp), ("u_init", _dp), ("u_nominal0", _dp),
                ("params", C.c_void_p), ("params_bytes", C.c_uint64), ("seed", C.c_uint64),
                ("device", C.c_int32), ("use_graph", C.c_int32), ("stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64), ("nu_diag", _dp),
                ("weighting", C.c_int32), ("kernels", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("hbm_budget_bytes", C.c_uint64), ("max_slots", C.c_int32),
                ("max_inflight", C.c_int32), ("max_batch", C.c_int32), ("mode", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("bytes_used", C.c_uint64), ("slots_used", C.c_int32), ("queued", C.c_int32),
                ("inflight", C.c_int32), ("requests_done", C.c_int64), ("batches", C.c_int64),
                ("mean_batch", C.c_double), ("rollout_steps_done", C.c_int64)]


class Info(C.Structure):
    _fields_ = [("rollout_lanes", C.c_int32), ("rollout_mode", C.c_int32), ("rollout_blocks", C.c_int32),
                ("update_chunk", C.c_int32), ("update_blocks", C.c_int32), ("noise_groups", C.c_int32),
                ("workspace_bytes", C.c_uint64)]


ROLLOUT_COST_TO_GO, ROLLOUT_CRASH, ROLLOUT_STEP_SPLIT, ROLLOUT_DIAGONAL, ROLLOUT_FUSED = 1, 2, 4, 8, 16

SERVE_BATCHED, SERVE_PLAIN, SERVE_BATCHED_GRAPH = 0, 1, 2

_lib = None


def load() -> C.CDLL:
    """Load libmppi.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1509_01149_amd.build.build() first")
    # One HIP runtime per process: PyTorch's ROCm wheel brings its own copy of the runtime,
    # so when torch is installed it is imported first and the library binds to that copy
    # (loaded the other way round, torch's later start-up finds no GPU).
    # MPPI_HIP_FROM_TORCH=0 skips it (processes that must not load torch).
    if os.environ.get("MPPI_HIP_FROM_TORCH", "1") != "0":
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    lib = C.CDLL(LIB_PATH)
    sig = {
        "mppi_workspace_bytes": [C.POINTER(Config), _u64p],
        "mppi_create": [C.POINTER(Config), C.POINTER(C.c_void_p)],
        "mppi_destroy": [C.c_void_p],
        "mppi_step": [C.c_void_p, _dp, C.c_int32, _dp],
        "mppi_step_static": [C.POINTER(Config), _dp, _dp, _u64p, C.c_int32, _dp],
        "mppi_step_async": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
        "mppi_step_plant_async": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
        "mppi_run_closed_loop_async": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p],
        "mppi_sync": [C.c_void_p],
        "mppi_plant_step_async": [C.c_void_p, C.c_void_p, C.c_void_p],
        "mppi_get_controls": [C.c_void_p, _dp, C.c_uint64],
        "mppi_set_controls": [C.c_void_p, _dp, C.c_uint64],
        "mppi_get_state": [C.c_void_p, C.c_void_p, C.c_uint64, _u64p],
        "mppi_set_state": [C.c_void_p, C.c_void_p, C.c_uint64],
        "mppi_get_iteration": [C.c_void_p, _u64p],
        "mppi_debug_last": [C.c_void_p, _dp, _dp, _dp, _dp],
        "mppi_debug_normals": [C.c_void_p, C.c_uint64, C.c_int32, C.c_int32, _fp],
        "mppi_debug_philox": [C.c_int32, C.c_uint64, _u32p, C.c_int32, _u32p],
        "mppi_debug_lane_groups": [C.c_int32, C.c_int32, _fp, _fp, C.c_int32, _fp],
        "mppi_set_profiling": [C.c_void_p, C.c_int32],
        "mppi_kernel_times": [C.c_void_p, _dp, C.POINTER(C.c_int64)],
        "mppi_get_info": [C.c_void_p, C.POINTER(Info)],
        "mppi_server_create": [C.POINTER(ServerConfig), C.POINTER(C.c_void_p)],
        "mppi_server_destroy": [C.c_void_p],
        "mppi_server_admit": [C.c_void_p, C.POINTER(Config), C.POINTER(C.c_int32)],
        "mppi_server_release": [C.c_void_p, C.c_int32],
        "mppi_server_submit": [C.c_void_p, C.c_int32, _dp, C.c_uint64, C.c_double],
        "mppi_server_poll": [C.c_void_p, C.c_int32, _u64p, _dp, C.POINTER(C.c_int32), _dp, C.POINTER(C.c_int32)],
        "mppi_server_replay": [C.c_void_p, C.c_int32, _dp, C.POINTER(C.c_int32), _dp, _dp, _dp,
                               C.POINTER(C.c_int32)],
        "mppi_server_replay_sessions": [C.c_void_p, C.c_int32, C.POINTER(Config), _dp, _dp, C.c_int32, _dp,
                                        C.POINTER(C.c_int32), _dp, _dp, _dp, C.POINTER(C.c_int32), _dp, _dp],
        "mppi_server_stats_get": [C.c_void_p, C.POINTER(ServerStats)],
        "mppi_server_get_controls": [C.c_void_p, C.c_int32, _dp, C.c_uint64],
        "mppi_mlp_create": [C.c_int32, _fp, C.POINTER(C.c_void_p)],
        "mppi_mlp_destroy": [C.c_void_p],
        "mppi_mlp_set_dataset": [C.c_void_p, C.POINTER(QuadrotorParams), C.c_double, _dp, _dp, C.c_int64],
        "mppi_mlp_get_targets": [C.c_void_p, _dp, C.c_int64],
        "mppi_mlp_set_stats": [C.c_void_p, _dp],
        "mppi_mlp_get_stats": [C.c_void_p, _dp],
        "mppi_mlp_get_params": [C.c_void_p, _fp],
        "mppi_mlp_set_params": [C.c_void_p, _fp],
        "mppi_mlp_train": [C.c_void_p, C.POINTER(C.c_int32), C.c_int64, C.c_int32, C.c_double, _dp],
        "mppi_mlp_loss_grads": [C.c_void_p, _dp, _dp, C.c_int32, _dp, _fp],
        "mppi_mlp_forward": [C.c_void_p, _dp, _dp, C.c_int32, _dp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.mppi_last_error.restype = C.c_char_p
    lib.mppi_last_error.argtypes = []
    lib.mppi_version.restype = C.c_char_p
    lib.mppi_version.argtypes = []
    lib.mppi_server_now.restype = C.c_double
    lib.mppi_server_now.argtypes = [C.c_void_p]
    _lib = lib
    return lib


def check(rc: int) -> int:
    if rc == OK:
        return rc
    msg = load().mppi_last_error().decode()
    if rc == ENUMERIC:
        raise NumericError(rc, msg)
    raise MppiError(rc, msg)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray], t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def make_params(system: int, params: Dict, keep: list):
    """Pack the system parameter dict (field names as in include/mppi.h) into its C struct."""
    if system == SYS_LINEAR:
        mats = [_f64(params[k]) for k in ("A", "B", "Q", "Qf")]
        keep.extend(mats)
        return LinearParams(*[_ptr(m) for m in mats])
    if system == SYS_CARTPOLE:
        p = CartPoleParams(params["mass_cart"], params["mass_pole"], params["half_length"], params["gravity"])
        p.q_diag[:] = list(_f64(params["q_diag"]))
        p.qf_diag[:] = list(_f64(params["qf_diag"]))
        return p
    if system == SYS_CARTPOLE_SWINGUP:
        return SwingUpParams(*[float(params[k]) for k in ("gain", "half_length", "gravity", "w_pos", "w_angle",
                                                           "w_vel", "w_rate")])
    if system == SYS_BICYCLE:
        m = np.ascontiguousarray(np.asarray(params["map"], dtype=np.float32))
        keep.append(m)
        return BicycleParams(params["wheelbase"], params["v_target"], params["w_speed"], params["cell_size"],
                             params["steer_limit"], m.shape[1], m.shape[0], _ptr(m, _fp))
    if system in (SYS_QUADROTOR, SYS_QUADROTOR_MLP):
        ob = _f64(params["obstacles"]).reshape(-1, 4)
        keep.append(ob)
        q = QuadrotorParams(params["mass"], params["gravity"], params["arm"], params["yaw_coef"])
        q.inertia[:] = list(_f64(params["inertia"]))
        q.goal[:] = list(_f64(params["goal"]))
        q.w_goal, q.w_obs, q.obs_margin = params["w_goal"], params["w_obs"], params["obs_margin"]
        q.n_obstacles = ob.shape[0]
        q.obstacles = _ptr(ob) if ob.shape[0] else None
        q.crash_cost, q.ground_z = float(params.get("crash_cost", 0.0)), float(params.get("ground_z", 0.0))
        if system == SYS_QUADROTOR:
            return q
        mlp = params["mlp"]
        keep.append(mlp)
        return QuadrotorMlpParams(q, C.c_void_p(mlp.handle.value))
    raise ValueError(f"unknown system {system}")


WEIGHT_PATH, WEIGHT_COST_TO_GO = 0, 1
KERNELS_AUTO, KERNELS_FUSED, KERNELS_THREE = 0, 2, 3


def make_config(*, system: int, n: int, m: int, K: int, T: int, dt: float, lam: float, nu,
                sigma, R=None, u_init, params: Dict, u_nominal0=None, seed: int = 0, device: int = 0,
                use_graph: bool = True, weighting: int = 0, kernels: int = 0):
    """Fill an mppi_config; returns (config, list of arrays that must stay alive)."""
    keep = []
    sig = _f64(sigma).reshape(m, m)
    Rm = None if R is None else _f64(R).reshape(m, m)
    ui = _f64(u_init).reshape(m)
    un = None if u_nominal0 is None else _f64(u_nominal0).reshape(T, m)
    nu_vec = None
    if np.ndim(nu) > 0:                 # per-dimension exploration factors
        nu_vec = _f64(nu).reshape(m)
        nu = float(nu_vec.max())
    keep += [sig, Rm, ui, un, nu_vec]
    prm = make_params(system, params, keep)
    keep.append(prm)
    cfg = Config()
    cfg.abi_version = ABI_VERSION
    cfg.system, cfg.n_state, cfg.n_ctrl, cfg.K, cfg.T = system, n, m, K, T
    cfg.dt, cfg.lambda_, cfg.nu = dt, lam, nu
    cfg.sigma, cfg.R, cfg.u_init, cfg.u_nominal0 = _ptr(sig), _ptr(Rm), _ptr(ui), _ptr(un)
    cfg.params = C.cast(C.pointer(prm), C.c_void_p)
    cfg.params_bytes = C.sizeof(prm)
    cfg.seed = seed & 0xFFFFFFFFFFFFFFFF
    cfg.device = device
    cfg.use_graph = 1 if use_graph else 0
    cfg.nu_diag = _ptr(nu_vec)
    cfg.weighting = weighting
    cfg.kernels = kernels
    return cfg, keep


STATIC_SCRATCH_BYTES = 8 << 20      # MPPI_STATIC_SCRATCH_BYTES


def step_static(x0, U, iteration: int, n_iters: int = 1, **config):
    """mppi_step_static: one control step without any device allocation, the controller state
    (nominal sequence U (T, m) and noise counter) held by the caller.  `config` takes the
    arguments of make_config.  Returns (u0, U after the update and the shift, iteration)."""
    lib = load()
    cfg, keep = make_config(**config)
    n, m, T = cfg.n_state, cfg.n_ctrl, cfg.T
    x = _f64(x0).reshape(n)
    Uc = _f64(U).reshape(T, m).copy()
    it = C.c_uint64(int(iteration))
    u0 = np.zeros(m)
    check(lib.mppi_step_static(C.byref(cfg), _ptr(x), _ptr(Uc), C.byref(it), int(n_iters), _ptr(u0)))
    return u0, Uc, int(it.value)


class Controller:
    """One MPPI controller context (mppi_create ... mppi_destroy)."""

    def __init__(self, *, system: int, n: int, m: int, K: int, T: int, dt: float, lam: float, nu,
                 sigma, R=None, u_init, params: Dict, u_nominal0=None, seed: int = 0, device: int = 0,
                 use_graph: bool = True, weighting: int = 0, kernels: int = 0, torch_stream=None,
                 torch_workspace: bool = False):
        lib = load()
        self.n, self.m, self.K, self.T = n, m, K, T
        cfg, self._keep = make_config(system=system, n=n, m=m, K=K, T=T, dt=dt, lam=lam, nu=nu, sigma=sigma, R=R,
                                      u_init=u_init, params=params, u_nominal0=u_nominal0, seed=seed,
                                      device=device, use_graph=use_graph, weighting=weighting, kernels=kernels)
        self._workspace = None
        if torch_stream is not None:
            cfg.stream = C.c_void_p(torch_stream.cuda_stream)
        if torch_workspace:
            import torch
            nbytes = C.c_uint64(0)
            check(lib.mppi_workspace_bytes(C.byref(cfg), C.byref(nbytes)))
            self._workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=f"cuda:{device}")
            base = self._workspace.data_ptr()
            cfg.workspace = C.c_void_p((base + 255) & ~255)
            cfg.workspace_bytes = nbytes.value
        self.cfg = cfg
        h = C.c_void_p()
        check(lib.mppi_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        self._lib = lib

    # -- control -----------------------------------------------------------------
    def step(self, x0, n_iters: int = 1) -> np.ndarray:
        """One control step from host state x0; returns u0 (m,)."""
        x = _f64(x0).reshape(self.n)
        u0 = np.zeros(self.m)
        check(self._lib.mppi_step(self.handle, _ptr(x), int(n_iters), _ptr(u0)))
        return u0

    def step_async(self, x0_dev_ptr: int, u0_dev_ptr: int, n_iters: int = 1):
        check(self._lib.mppi_step_async(self.handle, C.c_void_p(x0_dev_ptr), int(n_iters), C.c_void_p(u0_dev_ptr)))

    def step_plant_async(self, x_dev_ptr: int, u0_dev_ptr: int, n_iters: int = 1):
        """Device closed loop: step from x_dev, emit u0, then advance x_dev by the plant step."""
        check(self._lib.mppi_step_plant_async(self.handle, C.c_void_p(x_dev_ptr), int(n_iters), C.c_void_p(u0_dev_ptr)))

    def run_closed_loop_async(self, x_dev_ptr: int, n_steps: int, u_log_dev_ptr: int, n_iters: int = 1):
        """n_steps device closed-loop steps in one launch sequence; step j's u0 goes to
        u_log (device, n_steps x m FP64) row j."""
        check(self._lib.mppi_run_closed_loop_async(self.handle, C.c_void_p(x_dev_ptr), int(n_steps), int(n_iters),
                                                   C.c_void_p(u_log_dev_ptr)))

    def sync(self):
        check(self._lib.mppi_sync(self.handle))

    def plant_step_async(self, x_dev_ptr: int, u_dev_ptr: int):
        check(self._lib.mppi_plant_step_async(self.handle, C.c_void_p(x_dev_ptr), C.c_void_p(u_dev_ptr)))

    def get_controls(self) -> np.ndarray:
        u = np.zeros((self.T, self.m))
        check(self._lib.mppi_get_controls(self.handle, _ptr(u), u.size))
        return u

    def set_controls(self, U):
        u = _f64(U).reshape(self.T, self.m)
        check(self._lib.mppi_set_controls(self.handle, _ptr(u), u.size))

    def get_state(self) -> bytes:
        need = C.c_uint64(0)
        check(self._lib.mppi_get_state(self.handle, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        check(self._lib.mppi_get_state(self.handle, buf, need.value, C.byref(need)))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        check(self._lib.mppi_set_state(self.handle, buf, len(blob)))

    def iteration(self) -> int:
        v = C.c_uint64(0)
        check(self._lib.mppi_get_iteration(self.handle, C.byref(v)))
        return int(v.value)

    def debug_last(self):
        S = np.zeros(self.K)
        rho = C.c_double(0)
        eta = C.c_double(0)
        dU = np.zeros((self.T, self.m))
        check(self._lib.mppi_debug_last(self.handle, _ptr(S), C.byref(rho), C.byref(eta), _ptr(dU)))
        return S, rho.value, eta.value, dU

    def debug_normals(self, iteration: int, k0: int, nk: int) -> np.ndarray:
        out = np.zeros((nk, self.T, self.m), dtype=np.float32)
        check(self._lib.mppi_debug_normals(self.handle, int(iteration), int(k0), int(nk), _ptr(out, _fp)))
        return out

    def info(self) -> Dict:
        """The launch configuration this context chose (mppi_get_info)."""
        s = Info()
        check(self._lib.mppi_get_info(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Info._fields_}

    def set_profiling(self, on: bool):
        check(self._lib.mppi_set_profiling(self.handle, 1 if on else 0))

    def kernel_times(self):
        """Mean kernel durations (ms) and launch counts: {'rollout': (ms, n), 'update': ..., 'finalize': ...}."""
        avg = np.zeros(3)
        cnt = (C.c_int64 * 3)()
        check(self._lib.mppi_kernel_times(self.handle, _ptr(avg), cnt))
        return {k: (float(avg[i]), int(cnt[i])) for i, k in enumerate(("rollout", "update", "finalize"))}

    def close(self):
        if getattr(self, "handle", None):
            self._lib.mppi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Continuous-batching server (mppi_server_*)."""

    def __init__(self, *, device: int = 0, hbm_budget_bytes: int = 8 << 30, max_slots: int = 256,
                 max_inflight: int = 3, max_batch: int = 256, mode: int = SERVE_BATCHED):
        self._lib = load()
        cfg = ServerConfig(device, hbm_budget_bytes, max_slots, max_inflight, min(max_batch, max_slots), mode)
        h = C.c_void_p()
        check(self._lib.mppi_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        self.dims = {}

    def admit(self, **kw) -> int:
        """Admit a controller (keyword arguments as for Controller); returns its slot."""
        kw.pop("torch_stream", None)
        kw.pop("torch_workspace", None)
        cfg, keep = make_config(**kw)
        slot = C.c_int32(-1)
        check(self._lib.mppi_server_admit(self.handle, C.byref(cfg), C.byref(slot)))
        self.dims[slot.value] = (kw["n"], kw["m"], kw["T"], kw["K"])
        return slot.value

    def release(self, slot: int):
        check(self._lib.mppi_server_release(self.handle, slot))
        self.dims.pop(slot, None)

    def now(self) -> float:
        return self._lib.mppi_server_now(self.handle)

    def submit(self, slot: int, x0, req_id: int, t_arrival: Optional[float] = None):
        x = np.zeros(16)
        xv = _f64(x0).ravel()
        x[:xv.size] = xv
        t = self.now() if t_arrival is None else t_arrival
        check(self._lib.mppi_server_submit(self.handle, slot, _ptr(x), req_id, t))

    def poll(self, max_results: int = 1024):
        ids = np.zeros(max_results, dtype=np.uint64)
        u0 = np.zeros((max_results, 4))
        st = np.zeros(max_results, dtype=np.int32)
        td = np.zeros(max_results)
        n = C.c_int32(0)
        check(self._lib.mppi_server_poll(self.handle, max_results, _ptr(ids, _u64p), _ptr(u0),
                                         st.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(td), C.byref(n)))
        k = n.value
        return ids[:k], u0[:k], st[:k], td[:k]

    def replay(self, t_arrival, slots, x0s):
        """Real-time replay of an arrival trace; returns (t_done, u0s, status)."""
        t = _f64(t_arrival).ravel()
        sl = np.ascontiguousarray(np.asarray(slots, dtype=np.int32).ravel())
        n = t.size
        x = np.zeros((n, 16))
        x0s = np.asarray(x0s, dtype=np.float64).reshape(n, -1)
        x[:, :x0s.shape[1]] = x0s
        td = np.zeros(n)
        u0 = np.zeros((n, 4))
        st = np.zeros(n, dtype=np.int32)
        check(self._lib.mppi_server_replay(self.handle, n, _ptr(t), sl.ctypes.data_as(C.POINTER(C.c_int32)),
                                           _ptr(x), _ptr(td), _ptr(u0), st.ctypes.data_as(C.POINTER(C.c_int32))))
        return td, u0, st

    def replay_sessions(self, configs, t_start, t_end, t_arrival, sessions, x0s):
        """mppi_server_replay_sessions: controllers (keyword-argument dicts as for admit) that
        arrive at t_start, wait for admission by the HBM budget, serve their requests and leave
        after t_end.  Returns (t_done, u0s, status) per request and (t_admit, t_release) per
        session."""
        ns = len(configs)
        keep = []
        cfgs = (Config * ns)()
        for j, kw in enumerate(configs):
            kw = {k: v for k, v in kw.items() if k not in ("torch_stream", "torch_workspace")}
            cfg, kp = make_config(**kw)
            keep.append(kp)
            cfgs[j] = cfg
        ts, te = _f64(t_start).ravel(), _f64(t_end).ravel()
        t = _f64(t_arrival).ravel()
        sess = np.ascontiguousarray(np.asarray(sessions, dtype=np.int32).ravel())
        n = t.size
        x = np.zeros((n, 16))
        x0s = np.asarray(x0s, dtype=np.float64).reshape(n, -1)
        x[:, :x0s.shape[1]] = x0s
        td, u0, st = np.zeros(n), np.zeros((n, 4)), np.zeros(n, dtype=np.int32)
        ta, tr = np.zeros(ns), np.zeros(ns)
        i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        check(self._lib.mppi_server_replay_sessions(self.handle, ns, cfgs, _ptr(ts), _ptr(te), n, _ptr(t), i32(sess),
                                                    _ptr(x), _ptr(td), _ptr(u0), i32(st), _ptr(ta), _ptr(tr)))
        return td, u0, st, ta, tr

    def stats(self) -> Dict:
        s = ServerStats()
        check(self._lib.mppi_server_stats_get(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def get_controls(self, slot: int) -> np.ndarray:
        n, m, T, K = self.dims[slot]
        u = np.zeros((T, m))
        check(self._lib.mppi_server_get_controls(self.handle, slot, _ptr(u), u.size))
        return u

    def close(self):
        if getattr(self, "handle", None):
            self._lib.mppi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


MLP_PARAMS = 20236
MLP_STATS = 56
_MLP_SHAPES = [("W1", (128, 16)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("W3", (12, 128)), ("b3", (12,))]


def mlp_flatten(p: Dict) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate([np.asarray(p[k], np.float32).ravel() for k, _ in _MLP_SHAPES]))


def mlp_unflatten(flat: np.ndarray) -> Dict:
    out, o = {}, 0
    for k, shp in _MLP_SHAPES:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


class Mlp:
    """Learned dynamics network on the GPU (mppi_mlp_*): BF16 MFMA training and inference."""

    def __init__(self, params: Dict, device: int = 0):
        self._lib = load()
        flat = mlp_flatten(params)
        h = C.c_void_p()
        check(self._lib.mppi_mlp_create(device, _ptr(flat, _fp), C.byref(h)))
        self.handle = h
        self.n = 0

    def set_dataset(self, quad_params: Dict, dt: float, x, u):
        keep = []
        q = make_params(SYS_QUADROTOR, quad_params, keep)
        xv = _f64(x).reshape(-1, 12)
        uv = _f64(u).reshape(-1, 4)
        check(self._lib.mppi_mlp_set_dataset(self.handle, C.byref(q), dt, _ptr(xv), _ptr(uv), xv.shape[0]))
        self.n = xv.shape[0]

    def targets(self) -> np.ndarray:
        d = np.zeros((self.n, 12))
        check(self._lib.mppi_mlp_get_targets(self.handle, _ptr(d), self.n))
        return d

    def stats(self) -> np.ndarray:
        s = np.zeros(MLP_STATS)
        check(self._lib.mppi_mlp_get_stats(self.handle, _ptr(s)))
        return s

    def set_stats(self, stats):
        s = _f64(stats).ravel()
        check(self._lib.mppi_mlp_set_stats(self.handle, _ptr(s)))

    def params(self) -> Dict:
        f = np.zeros(MLP_PARAMS, dtype=np.float32)
        check(self._lib.mppi_mlp_get_params(self.handle, _ptr(f, _fp)))
        return mlp_unflatten(f)

    def set_params(self, params: Dict):
        f = mlp_flatten(params)
        check(self._lib.mppi_mlp_set_params(self.handle, _ptr(f, _fp)))

    def train(self, order, batch: int, lr: float) -> np.ndarray:
        o = np.ascontiguousarray(np.asarray(order, dtype=np.int32).ravel())
        steps = o.size // batch
        losses = np.zeros(steps)
        check(self._lib.mppi_mlp_train(self.handle, o.ctypes.data_as(C.POINTER(C.c_int32)), o.size, batch, lr,
                                       _ptr(losses)))
        return losses

    def loss_grads(self, zn, tn):
        z = _f64(zn).reshape(-1, 16)
        t = _f64(tn).reshape(-1, 12)
        loss = C.c_double(0)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        check(self._lib.mppi_mlp_loss_grads(self.handle, _ptr(z), _ptr(t), z.shape[0], C.byref(loss), _ptr(g, _fp)))
        return loss.value, mlp_unflatten(g)

    def forward(self, x, u) -> np.ndarray:
        xv = _f64(x).reshape(-1, 12)
        uv = _f64(u).reshape(-1, 4)
        dx = np.zeros((xv.shape[0], 12))
        check(self._lib.mppi_mlp_forward(self.handle, _ptr(xv), _ptr(uv), xv.shape[0], _ptr(dx)))
        return dx

    def close(self):
        if getattr(self, "handle", None):
            self._lib.mppi_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def philox(counters: np.ndarray, seed: int, device: int = 0) -> np.ndarray:
    """Raw Philox4x32-10 blocks computed on the GPU: counters (n, 4) uint32 -> (n, 4) uint32."""
    lib = load()
    c = np.ascontiguousarray(np.asarray(counters, dtype=np.uint32).reshape(-1, 4))
    out = np.zeros_like(c)
    check(lib.mppi_debug_philox(device, seed & 0xFFFFFFFFFFFFFFFF, _ptr(c, _u32p), c.shape[0], _ptr(out, _u32p)))
    return out


def lane_groups(a: np.ndarray, b: np.ndarray, group: int, device: int = 0) -> np.ndarray:
    """The rollouts' lane-group primitives on the GPU: a, b (64 n,) float32 -> (64 n, 6) float32
    (inclusive scan, exclusive scan, last-lane broadcast, group sum in the first lane,
    affine-scan slope and offset)."""
    lib = load()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).ravel())
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float32).ravel())
    if a.size != b.size or a.size % 64:
        raise ValueError("a and b must hold the same whole number of 64-lane waves")
    out = np.zeros((a.size, 6), dtype=np.float32)
    check(lib.mppi_debug_lane_groups(device, int(group), _ptr(a, _fp), _ptr(b, _fp), a.size // 64, _ptr(out, _fp)))
    return out


def version() -> str:
    return load().mppi_version().decode()
