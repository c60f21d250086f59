"""Pins of the oracle's Philox4x32-10 and of its noise draw (CPU only).

* the vectorised and the pure-Python implementations agree bit for bit;
* both agree with rocRAND's host-side Philox4x32-10, an implementation written by
  others from the same published definition (Salmon et al., SC'11);
* the uniforms and Box-Muller normals have the stated support and moments;
* one normal recomputed by hand from the counter layout matches the tensor entry;
* the exploration noise has covariance nu * Sigma and scales with sqrt(nu)
  (Section III-C: A = sqrt(nu) I).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import noise, philox

HERE = os.path.dirname(__file__)


def _random_blocks(n, seed=1):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    keys = rng.integers(0, 2 ** 64, size=n, dtype=np.uint64)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 0, 1]]
    keys[:4] = [0, 0xFFFFFFFFFFFFFFFF, 1, 1 << 32]
    return ctr, keys


def test_vectorised_matches_pure_python():
    ctr, keys = _random_blocks(300)
    k0, k1 = keys & np.uint64(0xFFFFFFFF), keys >> np.uint64(32)
    out = np.stack(philox.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], k0, k1), axis=1)
    for i in range(ctr.shape[0]):
        ref = philox.philox4x32_10_int(tuple(int(v) for v in ctr[i]), (int(k0[i]), int(k1[i])))
        assert tuple(int(v) for v in out[i]) == ref


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rocrand") / "ref")
    src = os.path.join(HERE, "golden", "rocrand_philox_ref.cpp")
    res = subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-x", "hip", src, "-o", exe],
                         capture_output=True, text=True)
    if res.returncode != 0:
        pytest.skip("could not build the rocRAND reference: " + res.stderr[-300:])
    return exe


def test_matches_rocrand_host_philox(rocrand_ref):
    ctr, keys = _random_blocks(200, seed=7)
    # rocRAND addresses blocks by a 64-bit offset counted in outputs (4 per block), so
    # counter word 1 must stay below 2^30 (the sample index k uses < 2^22).
    ctr[:, 1] &= np.uint64((1 << 30) - 1)
    lines = "\n".join(f"{c[0]} {c[1]} {c[2]} {c[3]} {k}" for c, k in zip(ctr, keys)) + "\n"
    res = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in ln.split()] for ln in res.stdout.strip().splitlines()], dtype=np.uint64)
    k0, k1 = keys & np.uint64(0xFFFFFFFF), keys >> np.uint64(32)
    out = np.stack(philox.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], k0, k1), axis=1)
    assert np.array_equal(out.astype(np.uint64), ref)


def test_uniforms_support():
    x = np.array([0, 255, 256, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    u = noise.uniforms_from_bits(x)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 2.0 ** -23
    assert u[3] == 1.0 and u[4] == 0.5 + 2.0 ** -24
    assert np.all((u > 0) & (u <= 1))
    assert np.all(u.astype(np.float32).astype(np.float64) == u)   # exact in FP32


def test_normals_moments_and_bound():
    e = noise.standard_normals(seed=3, iteration=11, K=4096, T=64, m=4).ravel()   # 1,048,576 draws
    n = e.size
    assert abs(e.mean()) < 5.0 / math.sqrt(n)
    assert abs(e.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    kurt = np.mean(e ** 4) / np.mean(e ** 2) ** 2
    assert abs(kurt - 3.0) < 5.0 * math.sqrt(24.0 / n)
    assert np.max(np.abs(e)) <= math.sqrt(48.0 * math.log(2.0)) + 1e-12
    # the two normals of one Box-Muller pair are uncorrelated
    pairs = noise.standard_normals(seed=3, iteration=11, K=4096, T=64, m=4).reshape(-1, 2)
    r = np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]
    assert abs(r) < 5.0 / math.sqrt(pairs.shape[0])


def test_counter_layout_by_hand():
    seed, it, K, T, m = 0x1234_5678_9ABC_DEF0, (1 << 33) + 5, 9, 7, 2
    e = noise.standard_normals(seed, it, K, T, m)
    k, i, j = 6, 5, 1
    f = i * m + j                                   # flat index 11 -> group 2, slot 3
    g, slot = divmod(f, 4)
    blk = philox.philox4x32_10_int((g, k, it & 0xFFFFFFFF, it >> 32), (seed & 0xFFFFFFFF, seed >> 32))
    ua = ((blk[2] >> 8) + 1) / 2 ** 24                # slot 3 is the sine of pair (2, 3)
    ub = ((blk[3] >> 8) + 1) / 2 ** 24
    want = math.sqrt(-2.0 * math.log(ua)) * math.sin(2.0 * math.pi * ub)
    assert slot == 3 and e[k, i, j] == pytest.approx(want, rel=1e-14, abs=1e-14)
    # a K offset addresses the same stream
    e2 = noise.standard_normals(seed, it, 3, T, m, k_offset=6)
    assert np.array_equal(e2[0], e[6])


def test_noise_covariance_is_nu_sigma():
    sigma = np.array([[0.5, 0.2], [0.2, 0.3]])
    nu = 3.0
    du = noise.control_noise(5, 0, 100_000, 4, sigma, nu).reshape(-1, 2)
    cov = np.cov(du.T)
    assert np.allclose(cov, nu * sigma, rtol=0.02, atol=0.01)
    du1 = noise.control_noise(5, 0, 50, 4, sigma, 1.0)
    du4 = noise.control_noise(5, 0, 50, 4, sigma, 4.0)
    assert np.allclose(du4, 2.0 * du1, rtol=1e-15, atol=0)
    # zero covariance: no noise at all
    assert not np.any(noise.control_noise(5, 0, 10, 4, np.zeros((2, 2)), 2.0))
