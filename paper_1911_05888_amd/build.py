"""Build the HIP library libldgs.so in-tree for gfx950.

Host setup code is compiled with g++ (OpenMP), the kernels with hipcc for
gfx950 only; the shared library is linked against the HIP runtime.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libldgs.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SRCS = ["setup.cpp", "build.cpp", "eigen.cpp", "rhs.cpp", "implicit.cpp", "api.cpp"]
HIP_SRCS = ["kernels.hip", "learned.hip", "setup_dev.hip", "implicit.hip"]

HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
               # no packed-FP32 instructions in generated code
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-munsafe-fp-atomics"]
GXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(ROCM, "include"), "-Wall", "-Wno-unused-function"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    inc = ["-I" + CSRC, "-I" + os.path.join(ROOT, "include")]
    for src in HIP_SRCS:
        obj = os.path.join(BUILD, src + ".o")
        _run([os.path.join(ROCM, "bin", "hipcc")] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    gxx = shutil.which("g++") or "g++"
    for src in HOST_SRCS:
        obj = os.path.join(BUILD, src + ".o")
        _run([gxx] + GXX_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([gxx, "-shared", "-o", tmp] + objs + ["-fopenmp", "-L" + os.path.join(ROCM, "lib"),
                                               "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
