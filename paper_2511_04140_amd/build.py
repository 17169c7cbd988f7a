"""Builds the HIP library libfalcon.so in-tree for gfx950.

All device code is compiled without FMA contraction, fast-math or
flush-to-zero (the codec's float arithmetic must match IEEE round-to-nearest
bit for bit) and with packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfalcon.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "api.cpp", "pipeline.cpp")]
ARCH = os.environ.get("FALCON_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS]
    for src in SOURCES:
        cmd += ["-x", "hip", src]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
