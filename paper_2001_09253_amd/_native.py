"""ctypes loader of the in-tree HIP library (libspline_solve.so).

There is no fallback: if the library is missing or does not load, every call
raises.  Build it with ``python -m paper_2001_09253_amd.build`` (or
``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os
import re
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspline_solve.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "spline_solve.h")

_lock = threading.Lock()
_lib = None

_vp = C.c_void_p
_d = C.c_double
_i64 = C.c_int64
_i32 = C.c_int32
_u32 = C.c_uint32
_u64 = C.c_uint64


class SolveConfig(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget_bytes", _u64), ("max_slots", _u32),
                ("precision", _u32), ("flags", _u32), ("max_inflight", _u32), ("stream", _vp)]


class Tuning(C.Structure):
    _fields_ = [("block", _i32), ("queries_per_tile", _i32), ("grid_per_cu", _i32), ("fused", _i32)]


SIGNATURES = {
    "solve_create": (C.c_int, [C.POINTER(SolveConfig), C.POINTER(_vp)]),
    "solve_submit": (C.c_int, [_vp, _vp, _vp, _i64, _d, _d, _vp, _i64, _vp, _vp, C.POINTER(_u64)]),
    "solve_poll": (C.c_int, [_vp, _u64, C.POINTER(C.c_int)]),
    "solve_wait": (C.c_int, [_vp, _u64, C.POINTER(C.c_int), _i64]),
    "solve_ticket_info": (C.c_int, [_vp, _u64, C.POINTER(_d), C.POINTER(C.c_int)]),
    "solve_clock": (_d, []),
    "solve_stats": (C.c_int, [_vp, C.POINTER(_u64)]),
    "solve_memory": (C.c_int, [_vp, C.POINTER(_u64)]),
    "solve_inject_fault": (C.c_int, [_vp]),
    "solve_destroy": (C.c_int, [_vp]),
    "spline_build": (C.c_int, [_vp, _vp, _i64, _d, _d, _vp, _vp, _vp]),
    "spline_solve_uniform": (C.c_int, [_vp, _vp, _i64, _d, _d, _i64, _vp, _vp, _vp, _vp]),
    "spline_solve_uniform_indexed": (C.c_int, [_vp, _vp, _i64, _d, _d, _i64, _vp, _vp, _vp, _vp, _vp]),
    "spline_solve_uniform_variant": (C.c_int, [_vp, _vp, _i64, _d, _d, _i64, _i32, _vp, _vp, _vp, _vp]),
    "spline_eval_uniform": (C.c_int, [_vp, _vp, _vp, _i64, _i64, _vp, _vp]),
    "spline_bracket_uniform": (C.c_int, [_vp, _i64, _i64, _vp, _vp]),
    "spline_noop_uniform": (C.c_int, [_vp, _i64, _i64, _vp, _vp]),
    "spline_eval_points": (C.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "spline_batch_eval_points": (C.c_int, [_i64, _i64] + [_vp] * 11),
    "spline_pack_knots": (C.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "spline_eval_points_packed": (C.c_int, [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "spline_plan_create": (C.c_int, [C.c_int, _i64, _vp, _vp, _u32, C.POINTER(Tuning), C.POINTER(_vp)]),
    "spline_plan_run": (C.c_int, [_vp] + [_vp] * 10),
    "spline_plan_run_indexed": (C.c_int, [_vp] + [_vp] * 11),
    "spline_plan_capture": (C.c_int, [_vp] + [_vp] * 10),
    "spline_plan_replay": (C.c_int, [_vp, _vp]),
    "spline_plan_autotune": (C.c_int, [_vp] + [_vp] * 8 + [C.c_int, C.c_char_p, C.POINTER(Tuning),
                                                          C.POINTER(_d)]),
    "spline_plan_get_tuning": (C.c_int, [_vp, C.POINTER(Tuning)]),
    "spline_plan_get_tables": (C.c_int, [_vp, _vp, _u64, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "spline_plan_destroy": (C.c_int, [_vp]),
    "spline_batch_run_noalloc": (C.c_int, [_i64, _vp, _vp, _u32, C.POINTER(Tuning)] + [_vp] * 10),
}


def header_functions():
    """Names of the functions include/spline_solve.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|double|uint64_t)\s+\**\s*(\w+)\s*\(", text)))


def lib():
    """The loaded library; raises if it is missing (no fallback path)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "HIP library %s is missing: build it with `python -m paper_2001_09253_amd.build`" % LIB_PATH)
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib
