"""Builds the HIP library ``libdpso.so`` in-tree for gfx950 with hipcc.

    python -m paper_1706_04399_amd.build          # compile (always rebuilds)
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdpso.so")
# memory-path micro-benchmarks for the benchmark's roofline report (not part of
# the DPSO library)
CEIL_SRC = os.path.join(PKG, "ceilings", "ceilings.hip")
CEIL_LIB = os.path.join(PKG, "libceilings.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the DPSO library)")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def command(out: str, srcs=None):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Wall", "-Wno-unused-result",
            # keep the compiler from forming packed fp32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC, "-o", out] + (srcs if srcs is not None else sources())


def _compile(lib: str, srcs, verbose: bool):
    tmp = lib + f".tmp{os.getpid()}"
    cmd = command(tmp, srcs)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed to build {os.path.basename(lib)}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    _compile(LIB, sources(), verbose)
    _compile(CEIL_LIB, [CEIL_SRC], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
