"""Builds liblbm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2604_13407_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(CSRC, n) for n in ("lbm_kernels.hip", "lbm_adjoint.hip", "lbm_static.hip", "lbm_api.cpp",
                                            "lbm_adjoint_api.cpp")]
HEADERS = [os.path.join(CSRC, n) for n in ("lbm_params.h", "lbm_node.h", "lbm_internal.h", "lbm_handle.h",
                                           "lbm_adjoint_node.h", "lbm_adjoint_internal.h")] + [
    os.path.join(ROOT, "include", "pplbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in generated device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # contraction of a*b+c into FMA only within one expression (as written), so that the
    # rounding of the step does not depend on how the optimiser shares or places code
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = True) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


C_CLIENT_SRC = os.path.join(ROOT, "tests", "c_client", "lbm_c_client.c")
C_CLIENT = os.path.join(HERE, "lbm_c_client")


def build_c_client(verbose: bool = True) -> str:
    """The plain-C client of the library (tests/c_client): gcc, C99, linked
    against liblbm.so beside it and the HIP runtime."""
    rocm = os.path.realpath(os.environ.get("ROCM_PATH", "/opt/rocm"))
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), C_CLIENT_SRC, "-o", C_CLIENT + ".tmp", "-L", HERE, "-llbm",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN",
           "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(C_CLIENT + ".tmp", C_CLIENT)
    return C_CLIENT


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    build()
    build_c_client()
    sys.exit(0)
