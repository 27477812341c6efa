"""The library's host code under AddressSanitizer: argument validation,
workspace layout, the low-rank factorisation and the C-ABI queries.  The
host-side tests run again, in a child process, against a build whose host
code is instrumented (the device code is not, and no kernel is launched).
CPU only."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_03296_amd", "csrc")


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def _build_host_asan(out: str) -> str:
    from paper_1511_03296_amd import build as B

    def compile_one(src: str) -> str:
        obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
        subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-O1", "-g", "-fPIC", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                        "-I" + B.INCLUDE, "-I" + CSRC, "-c", os.path.join(CSRC, src), "-o", obj],
                       check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = os.path.join(out, "libbsolve.so")
    subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-shared-libasan",
                    "-Xarch_host", "-fsanitize=address", "-o", lib, *objs],
                   check=True, capture_output=True)
    return lib


def test_host_code_under_address_sanitizer(tmp_path):
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("the clang AddressSanitizer runtime is not installed")
    lib = _build_host_asan(str(tmp_path))
    env = dict(os.environ, BSOLVE_LIB=lib, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          "tests/test_abi.py", "tests/test_lowrank_host.py"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in res.stdout
