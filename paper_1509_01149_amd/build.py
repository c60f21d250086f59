"""Build libmppi.so in-tree with hipcc for gfx950.

Usage: python -m paper_1509_01149_amd.build   (or build() from Python).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmppi.so")
SOURCES = ["mppi_api.hip", "mppi_server.hip", "mppi_mlp.hip"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # never emit packed FP32 instructions (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a*b + c only within one source expression, as the front end decides: every
    # kernel that runs the same code (fused or not, batched or not) rounds the same way
    "-ffp-contract=on",
    "-Wno-unused-result",
]
# Extra flags of one source.  The learned dynamics take their MFMA results in ordinary VGPRs
# (the VGPR form of the instruction) rather than in accumulation registers, so the rollout's
# activations are read without a copy out of them (same arithmetic; the rollout 3 % faster).
SOURCE_FLAGS = {
    "mppi_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libmppi")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}: {' '.join(cmd[-3:])}")


def build(verbose: bool = False, objdir: str = None) -> str:
    """Compile every source to an object in parallel, then link libmppi.so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = objdir or os.path.join(HERE, "_obj")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc(), *compile_flags, *SOURCE_FLAGS.get(s, []), "-I", os.path.join(HERE, "..", "include"), "-c",
             os.path.join(CSRC, s), "-o", o]
            for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(len(cmds)) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
