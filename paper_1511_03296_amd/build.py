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
           "bs_lowrank.hip", "bs_timing.hip", "bs_noalloc.hip", "bs_dt.hip"]

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
    _kernel_code([os.path.join(BUILD, "bs_solve.o"), os.path.join(BUILD, "bs_dt.o")])
    _build_example()
    if verbose:
        print("built", LIB)
    return LIB


KERNEL_CODE = os.path.join(PKG, "kernel_code.json")
LLVM = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin")


def _kernel_code(objs: list) -> None:
    """Writes kernel_code.json next to the library: a digest of the gfx950
    machine code of every kernel of the given objects (the solve and the
    domain-transform sources), by demangled name.
    Measurements taken on a kernel (bench.py's HBM traffic) stay valid while its
    digest is unchanged, whatever else in the source changes."""
    import hashlib
    import json
    import re
    tmp = os.path.join(BUILD, "kernel_code")
    os.makedirs(tmp, exist_ok=True)
    tool = lambda name: os.path.join(LLVM, name)
    out = {}
    for obj in objs:
        stem = os.path.splitext(os.path.basename(obj))[0]
        fb, co = os.path.join(tmp, stem + "_fatbin.bin"), os.path.join(tmp, stem + "_gfx950.o")
        subprocess.run([tool("llvm-objcopy"), f"--dump-section=.hip_fatbin={fb}", obj,
                        os.devnull], check=True, capture_output=True)
        subprocess.run([tool("clang-offload-bundler"), "--type=o", f"--input={fb}",
                        f"--output={co}", f"--targets=hipv4-amdgcn-amd-amdhsa--{ARCH}",
                        "--unbundle"], check=True, capture_output=True)
        data = open(co, "rb").read()
        secs = subprocess.run([tool("llvm-readelf"), "-S", "-W", co], check=True,
                              capture_output=True, text=True).stdout
        m = re.search(r"\]\s+\.text\s+PROGBITS\s+([0-9a-f]+)\s+([0-9a-f]+)", secs)
        base = int(m.group(2), 16) - int(m.group(1), 16)
        syms = subprocess.run([tool("llvm-readelf"), "-s", "-W", co], check=True,
                              capture_output=True, text=True).stdout
        funcs = []
        for line in syms.splitlines():
            f = line.split()
            if len(f) >= 8 and f[3] == "FUNC" and int(f[2]) > 0:
                start = base + int(f[1], 16)
                digest = hashlib.sha256(data[start:start + int(f[2])]).hexdigest()[:16]
                funcs.append((f[7], digest))
        names = subprocess.run(["c++filt"], input="\n".join(n for n, _ in funcs), check=True,
                               capture_output=True, text=True).stdout.splitlines()
        for (_, digest), name in zip(funcs, names):
            name = re.sub(r"^void ", "", name)
            out[re.sub(r"\(.*\)$", "", name)] = digest
    with open(KERNEL_CODE + ".tmp", "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    os.replace(KERNEL_CODE + ".tmp", KERNEL_CODE)


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
