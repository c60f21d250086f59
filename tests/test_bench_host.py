"""Host-side logic of bench.py, without a GPU: the one-GPU guard, the workloads it can
time and the per-workload operation counts its roofline line divides by."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

# the workloads bench.py times without training a network first: (name, K, T, m)
WORKLOADS = [("bicycle", 4096, 100, 2), ("bicycle_ctg", 4096, 100, 2), ("cartpole", 1000, 100, 1),
             ("quadrotor", 16384, 150, 4), ("quadrotor_crash", 16384, 150, 4), ("swingup", 4096, 50, 1)]


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("name,K,T,m", WORKLOADS)
def test_workloads_have_their_sizes_and_operation_counts(name, K, T, m):
    wl = bench.make_workload(name)
    assert (wl.K, wl.T, wl.m) == (K, T, m)
    assert bench.ALG_FLOP_PER_ROLLOUT_STEP[wl.name] > 0
    assert bench.ISSUE_OPS_PER_ROLLOUT_STEP[wl.name] >= bench.ALG_FLOP_PER_ROLLOUT_STEP[wl.name]


def test_unknown_workload_is_an_error():
    with pytest.raises(SystemExit):
        bench.make_workload("no_such_workload")


def test_peaks():
    # the published FP32 peak is the denominator of frac; the build's own unpacked-FP32 issue
    # ceiling is 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP per FMA x 2.4 GHz
    assert bench.FP32_PEAK_TFLOPS == 157.3
    assert abs(bench.ALU_PEAK_TFLOPS - 78.6432) < 1e-3


def test_default_workload_is_the_largest_single_gpu_configuration():
    import argparse
    wl = bench.make_workload("quadrotor")
    assert (wl.K, wl.T, wl.n, wl.m, wl.nu) == (16384, 150, 12, 4, 2.0)
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--workload", default="quadrotor")' in src


def test_sharded_oracle_equals_one_process():
    """The CPU leg's sharded oracle (K split into contiguous ranges, the shards' partial sums
    merged exactly) reproduces the one-process oracle's control step."""
    import numpy as np
    import workloads as W
    from oracle import mppi
    wl = W.bicycle(K=300, T=12).replace(seed=4)
    U = mppi.initial_sequence(wl) + 0.05
    bench._shard_init(wl)
    bounds = [0, 37, 150, 151, 300]
    parts = [bench._shard_partials((wl.x0, U, 3, bounds[g], bounds[g + 1])) for g in range(4)]
    dU = mppi.merge_shards(parts, wl.lam)
    ref = mppi.iteration(wl, wl.x0, U, 3)
    assert np.allclose(dU, ref.dU, rtol=1e-12, atol=1e-14)


def test_host_cores_is_bounded():
    assert 1 <= bench.host_cores() <= 16
