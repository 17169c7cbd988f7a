"""Builds the HIP library libfalcon.so in-tree for gfx950.

All device code is compiled without FMA contraction, fast-math or
flush-to-zero (the codec's float arithmetic must match IEEE round-to-nearest
bit for bit) and with packed FP32 instructions disabled.  Each source is
compiled to an object of its own, in parallel, then linked.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfalcon.so")
SOURCES = [os.path.join(CSRC, f) for f in (
    "kernels_f64.hip", "kernels_f32.hip", "kernels_mixed.hip", "kernels_common.hip", "noalloc.hip",
    "api.cpp", "pipeline.cpp", "batch.cpp", "serve.cpp")]
ARCH = os.environ.get("FALCON_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# Per-source additions.  The float32 kernels are built with uniform branches
# left unstructured: a wave-uniform if/else then compiles to one scalar
# branch instead of exec-mask bookkeeping (per bit-plane row in the payload
# assembly and the decoder).  Measured on MI355X: float32 compression 4.6 %
# and decoding 2.6 % faster; the float64 kernels measured 1-2 % slower and
# keep the default.
SOURCE_FLAGS = {
    "kernels_f32.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions=1"],
}


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        cmd = [hipcc, *FLAGS, *SOURCE_FLAGS.get(os.path.basename(src), []), "-c", "-x", "hip", src, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    workers = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
