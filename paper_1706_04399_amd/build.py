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


FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
         # keep the compiler from forming packed fp32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def command(out: str, srcs=None):
    """One hipcc line that compiles and links `srcs` into the shared library `out`."""
    return [hipcc()] + FLAGS + ["-shared", "-o", out] + (srcs if srcs is not None else sources())


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed to build {what}")


def _compile(lib: str, srcs, verbose: bool):
    """Each source to an object in parallel (one code object per source), then
    one link; the library replaces the old one only when the link succeeded."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(os.path.dirname(lib), "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = f".{os.getpid()}.o"
    objs = [os.path.join(objdir, os.path.basename(src) + tag) for src in srcs]
    jobs = max(1, min(len(srcs), os.cpu_count() or 1, 16))
    try:
        with ThreadPoolExecutor(jobs) as pool:
            list(pool.map(lambda so: _run([hipcc()] + FLAGS + ["-c", so[0], "-o", so[1]], so[0], verbose),
                          zip(srcs, objs)))
        tmp = lib + f".tmp{os.getpid()}"
        _run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs,
             os.path.basename(lib), verbose)
        os.replace(tmp, lib)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)


def build(verbose: bool = False) -> str:
    _compile(LIB, sources(), verbose)
    _compile(CEIL_LIB, [CEIL_SRC], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
