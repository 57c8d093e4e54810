"""Builds libegosgm.so, the HIP library behind include/egosgm.h, for gfx950.

Run as ``python -m paper_1708_06301_amd.build``; the library lands next to
this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(PKG, "libegosgm.so")
SOURCES = ["egosgm_kernels.hip", "egosgm_api.hip", "egosgm_vo.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # float32 steps that decide integers (warp target pixel, windows) must be
    # evaluated exactly as written: no contraction, correctly rounded / and sqrt
    "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    # never emit packed-fp32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", INCLUDE,
]


def build(verbose: bool = False) -> str:
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
