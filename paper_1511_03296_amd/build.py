"""Builds libbsolve.so, the HIP library of the bilateral solver, for gfx950.

Every call recompiles all sources (hipcc cross-compiles without a GPU):
    python -m paper_1511_03296_amd.build
Objects go to ``_build/`` at the repository root; the shared library is
written next to this file, where the binding loads it from.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbsolve.so")
SOURCES = ["bs_grid.hip", "bs_bistoch.hip", "bs_solve.hip", "bs_batch.hip", "bs_robust.hip",
           "bs_lowrank.hip", "bs_timing.hip"]

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 instructions are disabled: hand-written or compiler-formed
    # v_pk_* FP32 arithmetic is avoided on this target.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 5)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    _build_example()
    if verbose:
        print("built", LIB)
    return LIB


EXAMPLE = os.path.join(PKG, "examples", "solve_c")


def _build_example() -> None:
    """The C-ABI example program, linked against the library next to it."""
    src = EXAMPLE + ".cpp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-I" + INCLUDE, src, "-L" + PKG, "-lbsolve",
           "-Wl,-rpath,$ORIGIN/..", "-o", EXAMPLE + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"example build failed:\n{res.stdout}\n{res.stderr}")
    os.replace(EXAMPLE + ".tmp", EXAMPLE)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
