"""Build the gfx950 shared library of the ray tracer with hipcc.

    python -m paper_2605_05635_amd.build [--verbose]

Produces paper_2605_05635_amd/libgeodesic_rt.so from csrc/*.hip.  Always
recompiles.  The library exports the C ABI declared in include/rt.h.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libgeodesic_rt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code: the compiler
# never forms them from scalar float code with this feature turned off.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
# The trace kernels use ~100 distinct binary64 constants (integrator tableau,
# series coefficients).  Machine-level loop-invariant code motion hoists all
# of their materialisations out of the persistent ray loop, which overflows
# the scalar registers and spills them to vector-register lanes (one VALU
# read per use inside the loop).  Without that pass the constants are
# rematerialised by scalar moves next to their uses.
# Floating-point contraction only within one expression (the C rule): fused
# multiply-adds then depend on the source alone, not on the surrounding code,
# so the single-image and batched kernels round every ray identically.
CODEGEN_FLAGS = ["-mllvm", "-disable-machine-licm", "-ffp-contract=on"]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    srcs = sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))
    cmd = [HIPCC, *DEVICE_FLAGS, *CODEGEN_FLAGS, "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           *(extra or []), "-o", LIB + ".tmp", *srcs,
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="--verbose" in sys.argv)
