"""ctypes binding of libupsample.so (include/upsample.h).

Argument marshalling only: every step of the upsampling path runs in the HIP
library.  The library is loaded from this package directory; if it is missing
the import of the binding fails loudly (build it with
``python -m paper_2308_01629_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libupsample.so")

UPSAMPLE_OK = 0
ERR_NAMES = {
    1: "UPSAMPLE_ERR_INVALID_ARG", 2: "UPSAMPLE_ERR_CAPACITY", 3: "UPSAMPLE_ERR_GRID_TOO_LARGE",
    4: "UPSAMPLE_ERR_NO_DEVICE", 5: "UPSAMPLE_ERR_OOM", 6: "UPSAMPLE_ERR_HIP",
    7: "UPSAMPLE_ERR_NONFINITE", 8: "UPSAMPLE_ERR_STATE",
}
ERR_CODES = {v: k for k, v in ERR_NAMES.items()}
MAX_WALLS = 32
WALL_FLOATS = 12
DEFAULT_CELL_FACTOR = 1.0001
FLAG_VALIDATE = 1
FLAG_DETERMINISTIC_BWD = 2
NOALLOC_MAX_LR = 65536
NOALLOC_MAX_CELLS = 262144
BATCH_EAGER = 1
PBD_GRANULAR = -1
PBD_STATIC = -2


class UpsampleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("r_lr", ctypes.c_float), ("r_hr", ctypes.c_float), ("dt", ctypes.c_float),
        ("g", ctypes.c_float * 3), ("c1", ctypes.c_float), ("c2", ctypes.c_float),
        ("domain_lo", ctypes.c_float * 3), ("domain_hi", ctypes.c_float * 3),
        ("cell_factor", ctypes.c_float), ("n_walls", ctypes.c_int32),
        ("walls", ctypes.POINTER(ctypes.c_float)),
        ("max_lr", ctypes.c_int64), ("max_hr", ctypes.c_int64), ("flags", ctypes.c_uint32),
    ]


class PbdParams(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_float), ("dt", ctypes.c_float), ("g", ctypes.c_float * 3),
        ("mu_s", ctypes.c_float), ("mu_k", ctypes.c_float), ("ground_y", ctypes.c_float),
        ("stab_iters", ctypes.c_int32), ("solve_iters", ctypes.c_int32), ("mass_scaling", ctypes.c_int32),
        ("domain_lo", ctypes.c_float * 3), ("domain_hi", ctypes.c_float * 3),
        ("max_neighbors", ctypes.c_int32),
    ]


class GridInfo(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32 * 3), ("reach", ctypes.c_int32), ("n_cells", ctypes.c_int64),
        ("cell_size", ctypes.c_double), ("inv_cell_size", ctypes.c_float), ("h2", ctypes.c_float),
        ("inv_h2", ctypes.c_float), ("lo", ctypes.c_float * 3),
    ]

    def as_dict(self) -> dict:
        return {"dims": tuple(self.dims), "reach": int(self.reach), "n_cells": int(self.n_cells),
                "cell_size": float(self.cell_size), "inv_cell_size": float(self.inv_cell_size),
                "h2": float(self.h2), "inv_h2": float(self.inv_h2), "lo": tuple(self.lo)}


class Tuning(ctypes.Structure):
    _fields_ = [("gather_groups", ctypes.c_int32), ("sort_sub", ctypes.c_int32),
                ("adjoint_tiled", ctypes.c_int32), ("sort_mode", ctypes.c_int32),
                ("tile_max", ctypes.c_int32), ("adjoint_tile_max", ctypes.c_int32),
                ("wall_cull", ctypes.c_int32)]


class AutotuneResult(ctypes.Structure):
    _fields_ = [("cell_factor", ctypes.c_float), ("tuning", Tuning), ("advance_ms", ctypes.c_float),
                ("from_cache", ctypes.c_int32)]


class SceneDesc(ctypes.Structure):
    """upsample_scene: one scene of a batch."""
    _fields_ = [("params", Params), ("lr_offset", ctypes.c_int64), ("n_lr", ctypes.c_int64),
                ("hr_offset", ctypes.c_int64), ("n_hr", ctypes.c_int64)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_INT = ctypes.c_int

# name -> (restype, argtypes); mirrors include/upsample.h
SIGNATURES = {
    "upsample_default_params": (_INT, [ctypes.POINTER(Params)]),
    "upsample_grid_info_for": (_INT, [ctypes.POINTER(Params), ctypes.POINTER(GridInfo)]),
    "upsample_init": (_INT, [ctypes.POINTER(Params), ctypes.POINTER(_P)]),
    "upsample_destroy": (_INT, [_P]),
    "upsample_strerror": (ctypes.c_char_p, [_INT]),
    "upsample_last_error": (ctypes.c_char_p, [_P]),
    "upsample_get_grid_info": (_INT, [_P, ctypes.POINTER(GridInfo)]),
    "upsample_build_grid": (_INT, [_P, _P, _P, _P, _I64, _P]),
    "upsample_advance": (_INT, [_P, _P, _P, _P, _P, _I64, _P]),
    "upsample_step": (_INT, [_P, _P, _P, _P, _I64, _P, _P, _P, _P, _I64, _P]),
    "upsample_step_backward": (_INT, [_P, _P, _P, _P, _I64, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "upsample_step_taped": (_INT, [_P, _P, _P, _P, _I64, _P, _P, _P, _P, _I64, _P, _P]),
    "upsample_step_backward_taped": (_INT, [_P, _P, _P, _P, _I64, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P,
                                            _P]),
    "upsample_grid_snapshot_bytes": (_INT, [_P, ctypes.POINTER(_I64)]),
    "upsample_grid_snapshot": (_INT, [_P, _P, _P]),
    "upsample_step_backward_taped_grid": (_INT, [_P, _P, _P, _I64, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P,
                                                 _P]),
    "upsample_run": (_INT, [_P, _P, _P, _P, _I64, _I32, _P, _P, _I64, _I32, _P, _P]),
    "upsample_run_multirate": (_INT, [_P, _P, _P, _P, _I64, _I32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, _I32, _P, _P, _I64, _I32, _P, _P]),
    "upsample_debug_lr_sorted": (_INT, [_P, _P, _P, _P]),
    "upsample_sort_hr": (_INT, [_P, _P, _P, _P, _P, _I64, _P, _P]),
    "upsample_permute": (_INT, [_P, _P, _P, _P, _P, _I64, _P, _INT, _P]),
    "upsample_debug_grid": (_INT, [_P, _P, _P, _P, _P]),
    "upsample_debug_neighbors": (_INT, [_P, _P, _P, _I64, _P, _P, _I64, _P, _P]),
    "upsample_debug_step_members": (_INT, [_P, _P, _P, _P, _P, _I64, _P, _P, _I64, _P, _P, _P]),
    "upsample_set_tuning": (_INT, [_P, ctypes.POINTER(Tuning)]),
    "upsample_get_tuning": (_INT, [_P, ctypes.POINTER(Tuning)]),
    "upsample_timing_enable": (_INT, [_P, _INT]),
    "upsample_timing_read": (_INT, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "upsample_step_noalloc": (_INT, [ctypes.POINTER(Params), _P, _P, _P, _I64, _P, _P, _P, _P, _I64, _P]),
    "upsample_sample_volume": (_INT, [_P, _I64, ctypes.c_float, ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_float), _P, _I64, ctypes.POINTER(_I64), _P]),
    "upsample_pbd_default_params": (_INT, [ctypes.POINTER(PbdParams)]),
    "upsample_pbd_init": (_INT, [ctypes.POINTER(PbdParams), _I64, _P, _P, _P, ctypes.POINTER(_P)]),
    "upsample_pbd_step": (_INT, [_P, _P, _P, _I32, _P, _P, _P]),
    "upsample_pbd_status": (_INT, [_P, ctypes.POINTER(_I64), _P]),
    "upsample_pbd_info": (_INT, [_P, ctypes.POINTER(_I64)]),
    "upsample_pbd_debug_step": (_INT, [_P, _P, _P, _P, _I64, _P, _P, _P]),
    "upsample_pbd_destroy": (_INT, [_P]),
    "upsample_pbd_last_error": (ctypes.c_char_p, [_P]),
    "upsample_batch_init": (_INT, [ctypes.POINTER(SceneDesc), _I32, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "upsample_batch_step": (_INT, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "upsample_batch_sort_hr": (_INT, [_P, _P, _P, _P, _P]),
    "upsample_batch_destroy": (_INT, [_P]),
    "upsample_batch_last_error": (ctypes.c_char_p, [_P]),
    "upsample_batch_info": (_INT, [_P, ctypes.POINTER(_I64)]),
    "upsample_autotune": (_INT, [ctypes.POINTER(Params), _P, _P, _P, _I64, _I32, _P, _P, _I64, ctypes.c_char_p,
                                 _P, ctypes.POINTER(AutotuneResult)]),
}

_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2308_01629_amd.build` (the HIP path has no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, handle=None, last_error=None) -> None:
    if rc == UPSAMPLE_OK:
        return
    L = lib()
    msg = ""
    if handle is not None and last_error is not None:
        m = last_error(handle)
        msg = m.decode() if m else ""
    if not msg:
        msg = L.upsample_strerror(rc).decode()
    raise UpsampleError(rc, msg)
