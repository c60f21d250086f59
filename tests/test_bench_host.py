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
    assert bench.ALG_OPS_PER_ROLLOUT_STEP[wl.name] > 0


def test_unknown_workload_is_an_error():
    with pytest.raises(SystemExit):
        bench.make_workload("no_such_workload")


def test_alu_peak_is_the_unpacked_fp32_rate():
    # 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP per FMA x 2.4 GHz
    assert abs(bench.ALU_PEAK_TFLOPS - 78.6432) < 1e-3
