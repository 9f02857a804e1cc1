"""Compile the HIP library ``libmapcheck.so`` in-tree for gfx950.

Usage: ``python paper_0912_2555_amd/build.py``.  hipcc cross-compiles without a
GPU present.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "mapcheck.hip")
LIB = os.path.join(PKG, "libmapcheck.so")
ARCH = os.environ.get("MAPCHECK_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # No packed-FP32 instructions anywhere in this library.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# The measurement build: the same source with per-workgroup phase clocks in the
# loop kernel (map_phase_counters), loaded instead of the library only when
# MAPCHECK_LIB names it.
LIB_PHASES = os.path.join(PKG, "libmapcheck_phases.so")


def build(verbose: bool = False, phases: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = LIB_PHASES if phases else LIB
    tmp = lib + ".tmp"
    extra = ["-DMAPCHECK_PHASES"] if phases else []
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed to build {os.path.basename(lib)}")
    os.replace(tmp, lib)
    return lib


EXAMPLE_SRC = os.path.join(PKG, "examples", "detect.c")
EXAMPLE = os.path.join(PKG, "examples", "detect")


def build_example(verbose: bool = False) -> str:
    """The C usage example (plain C against the C ABI and the HIP runtime), linked to the built library."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = EXAMPLE + ".tmp"
    cmd = [os.environ.get("CC", "gcc"), "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"), EXAMPLE_SRC,
           "-L", PKG, "-lmapcheck", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("failed to build the C example")
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose=True))
    print(build(verbose=True, phases=True))
    print(build_example(verbose=True))
