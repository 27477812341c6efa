"""Host-side checks of the C ABI: the library loads, exports every function
include/bsolve.h declares, and rejects invalid arguments before touching the
GPU.  None of these tests launches a kernel."""
import ctypes as ct
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsolve.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(bs_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("bs_build_grid", "bs_bistochastize", "bs_solve", "bs_slice",
                 "bs_solve_backward", "bs_grid_workspace_bytes", "bs_solve_workspace_bytes"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_1511_03296_amd import _lib as L
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(bs_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(L.EXPORTED) == set(declared_functions())
    assert L.lib.bs_version() >> 16 == 1


def test_struct_sizes_match_header_layout():
    from paper_1511_03296_amd import _lib as L
    assert ct.sizeof(L.Grid) == L.BS_GRID_BYTES
    assert ct.sizeof(L.ChanStats) == 24
    assert ct.sizeof(L.SolveParams) == 48
    assert ct.sizeof(L.BistochParams) == 16


def test_workspace_queries_are_pure_and_validate():
    from paper_1511_03296_amd import _lib as L
    p = L.GridParams(8, 4, 4)
    n1 = L.lib.bs_grid_workspace_bytes(48, 64, ct.byref(p))
    n2 = L.lib.bs_grid_workspace_bytes(96, 128, ct.byref(p))
    assert n1 > 0 and n2 > n1 and n1 % 256 == 0
    assert L.lib.bs_grid_workspace_bytes(0, 64, ct.byref(p)) == 0
    assert L.lib.bs_grid_workspace_bytes(48, 64, ct.byref(L.GridParams(0, 4, 4))) == 0
    assert L.lib.bs_grid_workspace_bytes(48, 64, None) == 0


def test_invalid_arguments_are_rejected_before_launch():
    from paper_1511_03296_amd import _lib as L
    p = L.GridParams(8, 4, 4)
    g = L.Grid()
    st = L.lib.bs_build_grid(None, 48, 64, ct.byref(p), None, 0, None, ct.byref(g))
    assert st == L.BS_EINVAL and b"NULL" in L.lib.bs_last_error()
    st = L.lib.bs_build_grid(ct.c_void_p(256), 48, 64, ct.byref(p), ct.c_void_p(4096), 16, None,
                             ct.byref(g))
    assert st == L.BS_EWORKSPACE
    st = L.lib.bs_build_grid(ct.c_void_p(256), 48, 64, ct.byref(p), ct.c_void_p(4100), 1 << 40,
                             None, ct.byref(g))
    assert st == L.BS_EINVAL and b"aligned" in L.lib.bs_last_error()
    st = L.lib.bs_build_grid(ct.c_void_p(256), 70000, 64, ct.byref(p), ct.c_void_p(4096), 1 << 40,
                             None, ct.byref(g))
    assert st == L.BS_EUNSUPPORTED
    # a handle that was never built
    sp = L.SolveParams(1.0, 1, 25, 8, 0.0, 4.0, 0.0)
    st = L.lib.bs_solve(ct.byref(g), ct.c_void_p(256), ct.c_void_p(256), 1, ct.byref(sp),
                        ct.c_void_p(256), ct.c_void_p(4096), 1 << 30, None, None)
    assert st == L.BS_EINVAL and b"not built" in L.lib.bs_last_error()
    assert L.lib.bs_bistochastize(ct.byref(g), None, None) == L.BS_EINVAL
    assert L.lib.bs_slice(ct.byref(g), ct.c_void_p(256), 1, ct.c_void_p(256), None) == L.BS_EINVAL
    assert L.lib.bs_solve_workspace_bytes(ct.byref(g), 1) == 0
    assert L.lib.bs_robust_workspace_bytes(ct.byref(g), 1) == 0
    st = L.lib.bs_robust_solve(ct.byref(g), ct.c_void_p(256), ct.c_void_p(256), 1, ct.byref(sp),
                               1.0, 4, ct.c_void_p(256), ct.c_void_p(256), ct.c_void_p(4096),
                               1 << 30, None, None)
    assert st == L.BS_EINVAL
    assert L.lib.bs_status_string(L.BS_EWORKSPACE) == b"workspace too small"


def test_python_errors_map_statuses():
    from paper_1511_03296_amd import _lib as L
    L.lib.bs_build_grid(None, 48, 64, None, None, 0, None, None)
    with pytest.raises(ValueError):
        L.check(L.BS_EINVAL, "x")
    with pytest.raises(L.BsError):
        L.check(L.BS_EDEVICE, "x")


def test_batch_tuning_setters():
    from paper_1511_03296_amd import _lib as L
    assert [L.lib.bs_lane_width(c) for c in (1, 2, 3, 4, 5, 6, 21, 64, 0, 65)] == \
        [1, 2, 3, 4, 4, 3, 3, 4, 0, 0]
    assert L.lib.bs_batch_tiles_per_block(3) == 16 and L.lib.bs_batch_tiles_per_block(1) == 8
    assert L.lib.bs_batch_set_tiles_per_block(3, 4) == L.BS_OK
    assert L.lib.bs_batch_tiles_per_block(3) == 4
    assert L.lib.bs_batch_set_tiles_per_block(3, 0) == L.BS_OK
    assert L.lib.bs_batch_tiles_per_block(3) == 16
    assert L.lib.bs_batch_set_tiles_per_block(5, 4) == L.BS_EINVAL
    assert L.lib.bs_batch_set_tiles_per_block(2, 65) == L.BS_EINVAL
    assert L.lib.bs_batch_tiles_per_block(0) == 0


def test_ctypes_mirrors_match_the_c_layout(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets,
    as a C compiler lays them out (the library fills some of them, so a short
    mirror would be overrun)."""
    from paper_1511_03296_amd import _lib as L
    mirrors = {"bs_grid_params": L.GridParams, "bs_bistoch_params": L.BistochParams,
               "bs_solve_params": L.SolveParams, "bs_chan_stats": L.ChanStats,
               "bs_grid": L.Grid, "bs_grid_view": L.GridView, "bs_batch_item": L.BatchItem,
               "bs_dt_params": L.DtParams}
    c_name = {"lambda_": "lambda"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bsolve.h"',
             'int main(void) {']
    for cs, py in mirrors.items():
        lines.append(f'printf("{cs} size %zu\\n", sizeof({cs}));')
        for f in py._fields_:
            n = c_name.get(f[0], f[0])
            lines.append(f'printf("{cs} {f[0]} %zu\\n", offsetof({cs}, {n}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        cs, field, val = line.split()
        got[(cs, field)] = int(val)
    for cs, py in mirrors.items():
        assert got[(cs, "size")] == ct.sizeof(py), cs
        for f in py._fields_:
            assert got[(cs, f[0])] == getattr(py, f[0]).offset, (cs, f[0])


def test_image_size_limits():
    """Sides up to 65535 (16-bit key fields) and up to 2^30 pixels are sized;
    larger images are rejected by the pure workspace query."""
    from paper_1511_03296_amd import _lib as L
    p = L.GridParams(8, 4, 4)
    q = ct.byref(p)
    assert L.lib.bs_grid_workspace_bytes(1, 65535, q) > 0
    assert L.lib.bs_grid_workspace_bytes(65535, 1, q) > 0
    assert L.lib.bs_grid_workspace_bytes(1, 65536, q) == 0
    assert L.lib.bs_grid_workspace_bytes(65536, 1, q) == 0
    assert L.lib.bs_grid_workspace_bytes(32768, 32768, q) > 0      # exactly 2^30 pixels
    assert L.lib.bs_grid_workspace_bytes(32768, 32769, q) == 0


def test_domain_transform_arguments_are_rejected_before_launch():
    from paper_1511_03296_amd import _lib as L
    assert ct.sizeof(L.DtParams) == 12
    n = L.lib.bs_dt_workspace_bytes(48, 64)
    assert n >= 48 * 64 * 12 and n % 256 == 0
    assert L.lib.bs_dt_workspace_bytes(0, 64) == 0
    assert L.lib.bs_dt_workspace_bytes(70000, 4) == 0
    good = L.DtParams(8.0, 16.0, 3)
    dev, ws = ct.c_void_p(256), ct.c_void_p(1 << 20)

    def dt(ref=dev, H=48, W=64, x=dev, C=1, p=good, out=dev, w=ws, nb=n):
        return L.lib.bs_domain_transform(ref, H, W, x, C, ct.byref(p) if p else None, out, w,
                                         nb, None)
    assert dt(ref=None) == L.BS_EINVAL
    assert dt(p=None) == L.BS_EINVAL
    assert dt(p=L.DtParams(0.0, 16.0, 3)) == L.BS_EINVAL
    assert dt(p=L.DtParams(8.0, float("inf"), 3)) == L.BS_EINVAL
    assert dt(p=L.DtParams(8.0, 16.0, 0)) == L.BS_EINVAL
    assert dt(p=L.DtParams(8.0, 16.0, 17)) == L.BS_EINVAL
    assert dt(C=0) == L.BS_EINVAL and dt(C=65) == L.BS_EINVAL
    assert dt(x=ct.c_void_p(258)) == L.BS_EINVAL
    # partly overlapping input and output (x and out equal is allowed)
    assert dt(x=ct.c_void_p(256), out=ct.c_void_p(512)) == L.BS_EINVAL
    assert b"overlap" in L.lib.bs_last_error()
    assert dt(H=70000) == L.BS_EUNSUPPORTED
    assert dt(w=ct.c_void_p((1 << 20) + 4)) == L.BS_EINVAL
    assert dt(nb=n - 1) == L.BS_EWORKSPACE
    st = L.lib.bs_dt_confidence(dev, 48, 64, dev, ct.byref(good), 0.0, 0, dev, ws, n, None)
    assert st == L.BS_EINVAL and b"sigma_dt" in L.lib.bs_last_error()
    st = L.lib.bs_dt_confidence(dev, 48, 64, dev, ct.byref(good), 2.0, -1, dev, ws, n, None)
    assert st == L.BS_EINVAL


def test_autotuner_default_lane_rule_matches_the_library():
    from paper_1511_03296_amd import _lib as L, autotune
    for C in range(1, 65):
        assert L.lib.bs_set_lane_width(C, 0) == L.BS_OK
        assert autotune.lane_candidates_default(C) == L.lib.bs_lane_width(C), C
        assert autotune.lane_candidates_default(C) in autotune.lane_candidates(C)
