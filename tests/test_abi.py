"""The C ABI without a GPU: the library loads, exports every function include/mppi.h
declares, and rejects invalid configurations before touching a device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1509_01149_amd as P
import workloads as W
from paper_1509_01149_amd import binding as B

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|const char \*|void)\s+\*?(mppi_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "mppi_create" in names and "mppi_step" in names and "mppi_get_controls" in names
    lib = P.load()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mppi_\w+)", out))
    assert set(names) <= exported


def test_library_is_built_for_gfx950():
    out = subprocess.run(["strings", B.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


def _cfg(wl, **over):
    keep = []
    params = B.make_params(wl.system, wl.params, keep)
    sig = np.ascontiguousarray(wl.sigma, dtype=np.float64)
    R = np.ascontiguousarray(wl.R, dtype=np.float64)
    ui = np.ascontiguousarray(wl.u_init, dtype=np.float64)
    keep += [sig, R, ui, params]
    c = B.Config()
    c.abi_version = B.ABI_VERSION
    c.system, c.n_state, c.n_ctrl, c.K, c.T = wl.system, wl.n, wl.m, wl.K, wl.T
    c.dt, c.lambda_, c.nu = wl.dt, wl.lam, wl.nu
    c.sigma, c.R, c.u_init = B._ptr(sig), B._ptr(R), B._ptr(ui)
    c.params = C.cast(C.pointer(params), C.c_void_p)
    c.params_bytes = C.sizeof(params)
    for k, v in over.items():
        setattr(c, k, v)
    return c, keep


def _ws(c):
    n = C.c_uint64(0)
    rc = P.load().mppi_workspace_bytes(C.byref(c), C.byref(n))
    return rc, n.value


@pytest.mark.parametrize("make", [W.cartpole, W.bicycle, W.quadrotor, W.linear_double_integrator])
def test_valid_configs_size_their_workspace(make):
    wl = make()
    c, keep = _cfg(wl)
    rc, n = _ws(c)
    assert rc == B.OK and n >= wl.K * 8 + wl.T * wl.m * 12
    # more samples, more state (one kernel choice: AUTO may switch it with K)
    c, keep = _cfg(wl, kernels=B.KERNELS_THREE)
    c2, keep2 = _cfg(wl, K=wl.K * 2, kernels=B.KERNELS_THREE)
    assert _ws(c2)[1] > _ws(c)[1]


@pytest.mark.parametrize("field,value", [
    ("abi_version", 99), ("K", 0), ("K", (1 << 22) + 1), ("T", 0), ("T", 1025), ("n_state", 3),
    ("n_ctrl", 2), ("dt", 0.0), ("dt", float("nan")), ("lambda_", 0.0), ("lambda_", -1.0), ("nu", 0.0),
    ("system", 17), ("params_bytes", 8), ("sigma", None), ("u_init", None), ("params", None)])
def test_invalid_configs_are_rejected(field, value):
    c, keep = _cfg(W.cartpole(), **{field: value})
    rc, _ = _ws(c)
    assert rc == B.EINVAL
    assert len(P.load().mppi_last_error()) > 0


def test_sigma_must_be_positive_definite_and_symmetric():
    wl = W.bicycle()
    for bad in (np.array([[1.0, 2.0], [2.0, 1.0]]), np.array([[1.0, 0.1], [0.2, 1.0]]), np.array([[-1.0, 0], [0, 1.0]])):
        c, keep = _cfg(wl.replace(sigma=bad))
        assert _ws(c)[0] == B.EINVAL
    c, keep = _cfg(wl.replace(sigma=np.zeros((2, 2))))   # zero noise is allowed
    assert _ws(c)[0] == B.OK


def test_bicycle_map_and_quadrotor_obstacles_are_validated():
    wl = W.bicycle()
    c, keep = _cfg(wl.replace(params=dict(wl.params, map=np.zeros((1, 5), np.float32))))
    assert _ws(c)[0] == B.EINVAL
    q = W.quadrotor()
    c, keep = _cfg(q.replace(params=dict(q.params, obstacles=np.zeros((300, 4)))))
    assert _ws(c)[0] == B.EINVAL
    for bad in ([[1.0, np.nan, 1.0, 0.5]], [[1.0, 2.0, 1.0, -0.5]], [[1.0, 2.0, 1.0, 2e6]]):
        c, keep = _cfg(q.replace(params=dict(q.params, obstacles=np.array(bad))))
        assert _ws(c)[0] == B.EINVAL, bad
    c, keep = _cfg(q.replace(params=dict(q.params, obstacles=np.array([[1.0, 2.0, 1.0, 1e5]]))))
    assert _ws(c)[0] == B.OK
    c, keep = _cfg(q.replace(params=dict(q.params, w_obs=-1.0)))
    assert _ws(c)[0] == B.EINVAL
    c, keep = _cfg(q.replace(params=dict(q.params, mass=0.0)))
    assert _ws(c)[0] == B.EINVAL


def test_extension_fields_are_validated():
    """Per-dimension exploration factors, the weighting, the kernels choice, the crash
    indicator's parameters and the swing-up pole are checked before any device work."""
    wl = W.bicycle()
    bad_nu = np.array([1.0, 0.0])
    c, keep = _cfg(wl, nu_diag=B._ptr(bad_nu))
    assert _ws(c)[0] == B.EINVAL
    good_nu = np.array([1.0, 4.0])
    c, keep = _cfg(wl, nu_diag=B._ptr(good_nu))
    assert _ws(c)[0] == B.OK
    for over in (dict(weighting=2), dict(weighting=-1), dict(kernels=1), dict(kernels=4)):
        c, keep = _cfg(wl, **over)
        assert _ws(c)[0] == B.EINVAL, over
    # the fused iteration under path weighting: the step-split systems, and the quadrotor
    # (with or without the crash indicator) while a rollout block's normals fit the CU's LDS
    # (T = 153 with 32 obstacles is the longest horizon that does)
    for w, kernels, rc in ((wl, B.KERNELS_FUSED, B.OK), (wl, B.KERNELS_THREE, B.OK),
                           (W.quadrotor(), B.KERNELS_FUSED, B.OK), (W.quadrotor(), B.KERNELS_THREE, B.OK),
                           (W.quadrotor(T=153), B.KERNELS_FUSED, B.OK),
                           (W.quadrotor(T=154), B.KERNELS_FUSED, B.EINVAL),
                           (W.quadrotor(T=154), B.KERNELS_THREE, B.OK),
                           (W.quadrotor(crash=True), B.KERNELS_FUSED, B.OK),
                           (W.cartpole(), B.KERNELS_FUSED, B.OK)):
        c, keep = _cfg(w, kernels=kernels)
        assert _ws(c)[0] == rc, (w.name, w.T, kernels)
    # cost-to-go: fused on the step-split systems (running costs kept in LDS), not on the quadrotor
    c, keep = _cfg(wl, kernels=B.KERNELS_FUSED, weighting=B.WEIGHT_COST_TO_GO)
    assert _ws(c)[0] == B.OK
    c, keep = _cfg(W.quadrotor(), kernels=B.KERNELS_FUSED, weighting=B.WEIGHT_COST_TO_GO)
    assert _ws(c)[0] == B.EINVAL
    c, keep = _cfg(wl.replace(T=1024), kernels=B.KERNELS_FUSED, weighting=B.WEIGHT_COST_TO_GO)   # 66 KiB of running costs
    assert _ws(c)[0] == B.EINVAL
    c, keep = _cfg(wl.replace(K=1 << 20), kernels=B.KERNELS_FUSED)       # 16384 rollout blocks
    assert _ws(c)[0] == B.EINVAL
    # the three-kernel cost-to-go iteration keeps every sample's prefix costs [T][K] for the update
    c, keep = _cfg(wl, weighting=B.WEIGHT_COST_TO_GO, kernels=B.KERNELS_THREE)
    rc, n_ctg = _ws(c)
    c3, keep3 = _cfg(wl, kernels=B.KERNELS_THREE)
    n_three = _ws(c3)[1]
    assert rc == B.OK and n_ctg >= n_three + wl.T * wl.K * 8
    q = W.quadrotor(crash=True)
    c, keep = _cfg(q)
    assert _ws(c)[0] == B.OK
    c, keep = _cfg(q.replace(params=dict(q.params, crash_cost=-1.0)))
    assert _ws(c)[0] == B.EINVAL
    s = W.cartpole_swingup()
    c, keep = _cfg(s)
    assert _ws(c)[0] == B.OK
    c, keep = _cfg(s.replace(params=dict(s.params, half_length=0.0)))
    assert _ws(c)[0] == B.EINVAL


def test_create_needs_a_device_or_fails_cleanly():
    """Without a GPU, mppi_create reports MPPI_EDEVICE (never a silent CPU fallback)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.MppiError) as e:
        P.controller_for(W.cartpole())
    assert e.value.code == B.EDEVICE
    with pytest.raises(P.MppiError):
        P.philox(np.zeros((1, 4), np.uint32), 0)


def test_null_handles_are_rejected():
    lib = P.load()
    u = np.zeros(4)
    assert lib.mppi_step(None, B._ptr(u), 1, B._ptr(u)) == B.EINVAL
    assert lib.mppi_destroy(None) == B.OK


def test_auto_kernels_on_the_quadrotor_follow_the_block_count():
    """AUTO takes the fused quadrotor iteration while its rollout blocks (64 samples each)
    fit one per CU (256), the three-kernel one past that; the workspace shows which."""
    for K, fused in ((16384, True), (16385, False)):
        sizes = {}
        for kern in (B.KERNELS_AUTO, B.KERNELS_FUSED, B.KERNELS_THREE):
            c, keep = _cfg(W.quadrotor(K=K), kernels=kern)
            rc, n = _ws(c)
            assert rc == B.OK
            sizes[kern] = n
        assert sizes[B.KERNELS_FUSED] != sizes[B.KERNELS_THREE]
        assert sizes[B.KERNELS_AUTO] == sizes[B.KERNELS_FUSED if fused else B.KERNELS_THREE], (K, sizes)
