"""Compile the HIP sources into the in-tree shared library libimx.so (gfx950).

hipcc cross-compiles for gfx950 without a GPU present.  Packed FP32 code
generation is switched off for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libimx.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "api.cpp", "engine.cpp", "noalloc.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wall",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# Memory access-rate probe used by bench.py's calibration mode (not part of the method).
PROBE_LIB = os.path.join(PKG, "libimx_probe.so")
PROBE_SOURCES = [os.path.join(CSRC, "probe.hip")]


def _compile(out: str, sources, verbose: bool) -> None:
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _compile(LIB, SOURCES, verbose)
    _compile(PROBE_LIB, PROBE_SOURCES, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
