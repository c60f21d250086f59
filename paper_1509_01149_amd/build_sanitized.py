"""Build libmppi with AddressSanitizer and UndefinedBehaviorSanitizer on its host code (the
runtime's validation, layout, context, server and ctypes-facing paths), for CPU tests that
need no GPU.  The device code is compiled normally (sanitizers apply to the host pass only).

Usage: python -m paper_1509_01149_amd.build_sanitized
Run a program against it with the sanitizer runtime preloaded and the binding pointed at it:
  LD_PRELOAD=<asan_runtime()> MPPI_LIBRARY=<SAN_LIB> python ...
"""
import glob
import os
import subprocess
import sys

from .build import CSRC, HERE, SOURCES, hipcc

SAN_DIR = os.path.join(HERE, "_san")
SAN_LIB = os.path.join(SAN_DIR, "libmppi_san.so")
# host-pass sanitizers only: each -fsanitize= is scoped by the -Xarch_host before it
SAN_FLAGS = ("--offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -shared "
             "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
             "-Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined "
             "-Xclang -target-feature -Xclang -packed-fp32-ops -ffp-contract=on -Wno-unused-result").split()


def asan_runtime() -> str:
    """The shared AddressSanitizer runtime of the ROCm clang (to preload into Python)."""
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not c:
        raise RuntimeError("the clang AddressSanitizer runtime was not found under /opt/rocm/llvm")
    return c[-1]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def up_to_date() -> bool:
    if not os.path.exists(SAN_LIB) or not all(os.path.exists(o) for o in objects()):
        return False
    t = os.path.getmtime(SAN_LIB)
    deps = sources() + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(HERE, "..", "include", "mppi.h")]
    return all(os.path.getmtime(d) <= t for d in deps)


def objects():
    return [os.path.join(SAN_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]


def build_sanitized(verbose: bool = False) -> str:
    """Sanitized objects of every source (compiled in parallel), linked into SAN_LIB against
    the HIP runtime; the objects stay in SAN_DIR for other links (a runtime stand-in)."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(SAN_DIR, exist_ok=True)
    flags = [f for f in SAN_FLAGS if f != "-shared"]
    inc = ["-I", os.path.join(HERE, "..", "include")]
    cmds = [[hipcc(), *flags, *inc, "-c", src, "-o", obj] for src, obj in zip(sources(), objects())]

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc (sanitizer build) failed with exit code {res.returncode}")

    with ThreadPoolExecutor(len(cmds)) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    tmp = SAN_LIB + ".tmp"
    run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
         "-Xarch_host", "-fsanitize=undefined", *objects(), "-o", tmp])
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build_sanitized(verbose=True))
