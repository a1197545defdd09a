"""Build libllama.so (HIP for gfx950 + host C++) in-tree with hipcc.

    python -m paper_2102_01887_amd.build

Always recompiles.  Objects go to paper_2102_01887_amd/_build/, the shared
library to paper_2102_01887_amd/libllama.so.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libllama.so")

ARCH = "gfx950"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + INCLUDE, "-I" + CSRC]

KERNELS = ["llama_kernels.hip", "surrogate_kernels.hip", "sort_kernels.hip", "alpha_kernels.hip", "noalloc.hip", "sim_kernels.hip"]
HOST = ["llama_host.cpp", "surrogate_host.cpp", "serve_host.cpp", "next_host.cpp", "feedback_host.cpp"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in KERNELS:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        _run([HIPCC, "--offload-arch=" + ARCH, *COMMON, *DEVICE_FLAGS, "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in HOST:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        _run([HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON, "-fopenmp", "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-fopenmp", "-pthread", *objs, "-o", tmp,
          "-Wl,-rpath,/opt/rocm/lib:/opt/rocm/llvm/lib"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
