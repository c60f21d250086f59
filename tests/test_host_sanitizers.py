"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): the
ABI tests (validation of every configuration field, system parameters, null handles, the
no-device failure path) run in a child Python process against the sanitizer build of the
library, and any sanitizer report fails the run."""
import os
import subprocess
import sys

import pytest

from paper_1509_01149_amd import build_sanitized as S

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


@pytest.fixture(scope="module")
def san_lib():
    if not S.up_to_date():
        S.build_sanitized()
    return S.SAN_LIB


def test_abi_tests_pass_under_address_and_undefined_behaviour_sanitizers(san_lib):
    env = dict(os.environ, LD_PRELOAD=S.asan_runtime(), MPPI_LIBRARY=san_lib, MPPI_HIP_FROM_TORCH="0",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the library must not be loaded from the default path in the child
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:xdist", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py"), "-k", "not built_for_gfx950"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
    assert res.returncode == 0, out[-3000:]
    assert " passed" in out


def _mock_library():
    """libmppi's sanitized objects linked to the HIP stand-in instead of the HIP runtime."""
    mock_src = os.path.join(ROOT, "tests", "host_mock", "hip_mock.cpp")
    mock_obj = os.path.join(S.SAN_DIR, "hip_mock.o")
    lib = os.path.join(S.SAN_DIR, "libmppi_mock.so")
    clang = "/opt/rocm/llvm/bin/clang++"
    subprocess.run([clang, "-std=c++17", "-fPIC", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
                    "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c", mock_src, "-o", mock_obj], check=True)
    subprocess.run([clang, "-shared", "-fsanitize=address", *S.objects(), mock_obj, "-o", lib], check=True)
    return lib


def test_serving_host_logic_at_bench_scale_under_address_sanitizer(san_lib):
    """The serving runtime's host logic with 256 controllers, in every batching mode, through the
    pre-admitted replay and the session replay under a binding HBM budget, with AddressSanitizer
    on and device memory that faults on any host access (the HIP stand-in): no host memory
    error, no host dereference of device memory, every request served, every session admitted
    and released."""
    lib = _mock_library()
    env = dict(os.environ, LD_PRELOAD=S.asan_runtime(), MPPI_LIBRARY=lib, MPPI_HIP_FROM_TORCH="0",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_mock", "serve_at_scale.py"), ROOT, "1.5"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert "ERROR: AddressSanitizer" not in out
    assert res.returncode == 0 and out.strip().endswith("done"), out[-3000:]
