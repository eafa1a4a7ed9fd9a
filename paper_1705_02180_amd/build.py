"""Build libscps.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libscps.so")
SOURCES = [os.path.join(CSRC, f) for f in ("scps_kernels.hip", "scps_maps.hip", "scps_funnel.hip", "scps_api.cpp")]
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # hardware float64 atomics on coarse-grained device memory
    "-munsafe-fp-atomics",
    # no packed FP32 arithmetic: the compiler must not form v_pk_* float ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    cmd = ["hipcc", *FLAGS, "-I", INCLUDE, "-o", LIB, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
