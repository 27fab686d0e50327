"""Build librl.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_1304_7211_amd.build      (or __graft_entry__.build())

Always compiles (no staleness check): the caller decides when to build.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librl.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are switched off for all device code (some v_pk_* FP32 forms
# have been seen to give wrong results without any error); the host pass warns that it
# does not know the feature, which is harmless.
# The matrix-core kernel's accumulators are kept in ordinary VGPRs (the VGPR form of the
# MFMA instructions): with accumulation registers the compiler copied every accumulator
# between the two register files on each PSF line.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-mfma-vgpr-form=1",
         "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]
SOURCES = [os.path.join(CSRC, "rl_api.hip"), os.path.join(CSRC, "psf_compile.cpp")]


def build(verbose=False):
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC] + FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building librl.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
