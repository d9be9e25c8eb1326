"""Build libtnep.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2312_05233_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtnep.so")
SOURCES = ["api.hip", "eval_runtime.hip", "kernels_neighbors.hip", "kernels_eval.hip", "kernels_spectrum.hip",
           "spectra_api.hip", "population_api.hip", "model_file.hip", "server.hip", "noalloc_api.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-pthread",
]


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


HOST_CHECK = os.path.join(HERE, "_host_check.so")


def build_host_check(verbose: bool = True) -> str:
    """Host-only build of the descriptor arithmetic (csrc/tnep_math.h) used by
    the CPU self-check tests; not part of libtnep."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = HOST_CHECK + ".tmp"
    cmd = [hipcc, "-O2", "-fPIC", "-shared", "-o", tmp, os.path.join(CSRC, "host_check.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, HOST_CHECK)
    return HOST_CHECK


if __name__ == "__main__":
    build()
    build_host_check()
    sys.exit(0)
