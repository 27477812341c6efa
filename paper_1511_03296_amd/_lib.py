"""ctypes binding of libbsolve.so (the C ABI declared in include/bsolve.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Importing this module loads the library and fails loudly if it is missing.
BSOLVE_LIB, if set, names another build of the same library to load (the
host-sanitizer build of the tests).
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BSOLVE_LIB") or os.path.join(_HERE, "libbsolve.so")

BS_OK, BS_EINVAL, BS_EWORKSPACE, BS_EDEVICE, BS_EUNSUPPORTED = 0, -1, -2, -3, -4
BS_MAX_CHANNELS = 64
BS_MAX_LEVELS = 24
BS_GRID_BYTES = 4096
BS_INIT_FLAT, BS_INIT_HIER = 0, 1
BS_PRECOND_JACOBI, BS_PRECOND_HIER = 0, 1
BS_NOALLOC_SCRATCH_BYTES = 64 << 20

# Slots of the device counter array.
CNT_V, CNT_K, CNT_BIST_ITERS, CNT_BIST_DONE, CNT_BIST_SRC, CNT_LEVEL0 = 0, 1, 2, 3, 4, 8

REASONS = {0: "running", 1: "tolerance", 2: "max_iters", 3: "rho_zero", 4: "breakdown", 5: "b_zero"}


class GridParams(ct.Structure):
    _fields_ = [("sigma_xy", ct.c_int32), ("sigma_l", ct.c_int32), ("sigma_uv", ct.c_int32)]


class BistochParams(ct.Structure):
    _fields_ = [("max_iters", ct.c_int32), ("check_every", ct.c_int32), ("tol", ct.c_double)]


class SolveParams(ct.Structure):
    _fields_ = [("lambda_", ct.c_float), ("init", ct.c_int32), ("max_iters", ct.c_int32),
                ("check_every", ct.c_int32), ("rel_tol", ct.c_double),
                ("init_alpha", ct.c_float), ("init_beta", ct.c_float),
                ("precond", ct.c_int32), ("pre_alpha", ct.c_float), ("pre_beta", ct.c_float)]


class DtParams(ct.Structure):
    _fields_ = [("sigma_s", ct.c_float), ("sigma_r", ct.c_float), ("iters", ct.c_int32)]


class ChanStats(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("reason", ct.c_int32), ("rel_residual", ct.c_double),
                ("bnorm", ct.c_double)]


class Grid(ct.Structure):
    _fields_ = [("opaque", ct.c_uint64 * (BS_GRID_BYTES // 8))]


class GridView(ct.Structure):
    _fields_ = [
        ("H", ct.c_int32), ("W", ct.c_int32), ("P", ct.c_int32), ("levels", ct.c_int32),
        ("ncells_x", ct.c_int32), ("ncells_y", ct.c_int32), ("vcap", ct.c_int64),
        ("counts", ct.c_void_p), ("bist_residual", ct.c_void_p), ("key", ct.c_void_p),
        ("idx", ct.c_void_p), ("m", ct.c_void_p), ("nbr", ct.c_void_p),
        ("pix_ptr", ct.c_void_p), ("pix_list", ct.c_void_p), ("n", ct.c_void_p),
        ("nf", ct.c_void_p), ("nn", ct.c_void_p),
        ("level_cap", ct.c_int64 * BS_MAX_LEVELS),
        ("level_key", ct.c_void_p * BS_MAX_LEVELS),
        ("parent", ct.c_void_p * BS_MAX_LEVELS),
        ("ones", ct.c_void_p * BS_MAX_LEVELS),
        ("nb16", ct.c_void_p), ("nb_packed", ct.c_int32),
    ]


class BatchItem(ct.Structure):
    _fields_ = [("ref", ct.c_void_p), ("target", ct.c_void_p), ("conf", ct.c_void_p),
                ("H", ct.c_int32), ("W", ct.c_int32), ("C", ct.c_int32),
                ("sigma", GridParams), ("grid_ws", ct.c_void_p), ("grid_ws_bytes", ct.c_size_t),
                ("y", ct.c_void_p), ("x", ct.c_void_p), ("grad_x", ct.c_void_p),
                ("grad_t", ct.c_void_p), ("grad_c", ct.c_void_p), ("stats", ct.c_void_p)]


class BsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1511_03296_amd.build`")
    return ct.CDLL(LIB_PATH)


lib = _load()

_vp, _i32, _sz = ct.c_void_p, ct.c_int32, ct.c_size_t
_SIGS = {
    "bs_grid_workspace_bytes": (_sz, [_i32, _i32, ct.POINTER(GridParams)]),
    "bs_build_grid": (_i32, [_vp, _i32, _i32, ct.POINTER(GridParams), _vp, _sz, _vp,
                             ct.POINTER(Grid)]),
    "bs_bistochastize": (_i32, [ct.POINTER(Grid), ct.POINTER(BistochParams), _vp]),
    "bs_solve_workspace_bytes": (_sz, [ct.POINTER(Grid), _i32]),
    "bs_solve": (_i32, [ct.POINTER(Grid), _vp, _vp, _i32, ct.POINTER(SolveParams), _vp, _vp,
                        _sz, _vp, _vp]),
    "bs_solve_noalloc": (_i32, [ct.POINTER(Grid), _vp, _vp, _i32, ct.POINTER(SolveParams), _vp,
                                _vp, _vp]),
    "bs_slice": (_i32, [ct.POINTER(Grid), _vp, _i32, _vp, _vp]),
    "bs_robust_workspace_bytes": (_sz, [ct.POINTER(Grid), _i32]),
    "bs_lowrank_workspace_bytes": (_sz, [ct.POINTER(Grid), _i32]),
    "bs_solve_lowrank": (_i32, [ct.POINTER(Grid), _vp, _vp, _i32, ct.POINTER(SolveParams),
                                ct.c_double, _vp, _vp, _sz, _vp, ct.POINTER(_i32), _vp]),
    "bs_lowrank_factor": (_i32, [_vp, _i32, ct.c_double, _vp, _vp, ct.POINTER(_i32)]),
    "bs_robust_solve": (_i32, [ct.POINTER(Grid), _vp, _vp, _i32, ct.POINTER(SolveParams), ct.c_float,
                               _i32, _vp, _vp, _vp, _sz, _vp, _vp]),
    "bs_solve_backward": (_i32, [ct.POINTER(Grid), _vp, _vp, _vp, _vp, _i32,
                                 ct.POINTER(SolveParams), _vp, _vp, _vp, _vp, _sz, _vp, _vp]),
    "bs_read_counters": (_i32, [ct.POINTER(Grid), ct.POINTER(_i32), _i32, _vp]),
    "bs_grid_vertex_count": (_i32, [ct.POINTER(Grid), ct.POINTER(_i32), _vp]),
    "bs_grid_get_view": (_i32, [ct.POINTER(Grid), ct.POINTER(GridView)]),
    "bs_solve_channel_stride": (_i32, [_i32]),
    "bs_solve_ws_view": (_i32, [ct.POINTER(Grid), _i32, _vp, _sz, ct.POINTER(_vp),
                                ct.POINTER(_vp), ct.POINTER(_vp), ct.POINTER(_vp)]),
    "bs_batch_plan_workspace_bytes": (_sz, [ct.POINTER(BatchItem), _i32]),
    "bs_batch_plan_create": (_i32, [ct.POINTER(BatchItem), _i32, ct.POINTER(SolveParams),
                                    ct.POINTER(SolveParams), ct.POINTER(BistochParams), _vp, _sz,
                                    _vp, ct.POINTER(_vp)]),
    "bs_batch_run_forward": (_i32, [_vp, _vp]),
    "bs_batch_run_backward": (_i32, [_vp, _vp]),
    "bs_batch_plan_grid": (_i32, [_vp, _i32, ct.POINTER(Grid)]),
    "bs_batch_plan_destroy": (None, [_vp]),
    "bs_batch_workspace_bytes": (_sz, [ct.POINTER(BatchItem), _i32, _i32]),
    "bs_batch_forward": (_i32, [ct.POINTER(BatchItem), _i32, ct.POINTER(SolveParams),
                                ct.POINTER(BistochParams), ct.POINTER(Grid), _i32, _vp, _sz, _vp]),
    "bs_batch_backward": (_i32, [ct.POINTER(BatchItem), _i32, ct.POINTER(Grid),
                                 ct.POINTER(SolveParams), _i32, _vp, _sz, _vp]),
    "bs_batch_lowrank_workspace_bytes": (_sz, [ct.POINTER(BatchItem), _i32, _i32]),
    "bs_batch_set_tiles_per_block": (_i32, [_i32, _i32]),
    "bs_batch_tiles_per_block": (_i32, [_i32]),
    "bs_lane_width": (_i32, [_i32]),
    "bs_set_lane_width": (_i32, [_i32, _i32]),
    "bs_batch_forward_lowrank": (_i32, [ct.POINTER(BatchItem), _i32, ct.POINTER(SolveParams),
                                        ct.POINTER(BistochParams), ct.POINTER(Grid), _i32,
                                        ct.c_double, ct.POINTER(_i32), _vp, _sz, _vp]),
    "bs_dt_workspace_bytes": (_sz, [_i32, _i32]),
    "bs_domain_transform": (_i32, [_vp, _i32, _i32, _vp, _i32, ct.POINTER(DtParams), _vp, _vp,
                                   _sz, _vp]),
    "bs_dt_confidence": (_i32, [_vp, _i32, _i32, _vp, ct.POINTER(DtParams), ct.c_float, _i32,
                                _vp, _vp, _sz, _vp]),
    "bs_timing_enable": (_i32, [_i32]),
    "bs_timing_reset": (_i32, []),
    "bs_timing_read": (_i32, [ct.c_char_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)]),
    "bs_status_string": (ct.c_char_p, [_i32]),
    "bs_last_error": (ct.c_char_p, []),
    "bs_version": (_i32, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def check(status: int, where: str) -> None:
    """Raise on a non-OK status: ValueError for invalid arguments, BsError otherwise."""
    if status == BS_OK:
        return
    detail = lib.bs_last_error().decode()
    if status == BS_EINVAL:
        raise ValueError(f"{where}: {detail}")
    raise BsError(status, where, detail)
