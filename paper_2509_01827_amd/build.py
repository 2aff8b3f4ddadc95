"""Build libmct2d.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2509_01827_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libmct2d.so")
SOURCES = [os.path.join(CSRC, "mct2d_api.cpp"), os.path.join(CSRC, "mct2d_step.hip"),
           os.path.join(CSRC, "mct2d_screen.hip"), os.path.join(CSRC, "mct2d_state.hip"),
           os.path.join(CSRC, "mct2d_tri.hip"), os.path.join(CSRC, "mct2d_tri_host.cpp"),
           os.path.join(CSRC, "mct2d_tri_geom.hip")]
HEADERS = [os.path.join(CSRC, "mct2d_impl.h"), os.path.join(CSRC, "mct2d_device.h"),
           os.path.join(CSRC, "mct2d_tri.h"), os.path.join(CSRC, "mct2d_tri_host.h"),
           os.path.join(ROOT, "include", "mct2d.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # binary64 results must not depend on the compiler's contraction choices
    "-ffp-contract=off",
    # no packed FP32 instructions on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
