"""ctypes mirror of include/rayramses.h (argument marshalling only).

Loads the in-tree ``librayramses.so``.  There is no fallback: if the library
is missing the import fails with instructions to build it.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librayramses.so")

RR_OK = 0
STATUS_NAMES = {0: "RR_OK", -1: "RR_ERR_INVALID_ARG", -2: "RR_ERR_UNSUPPORTED", -3: "RR_ERR_OOM",
                -4: "RR_ERR_HIP", -5: "RR_ERR_OCTREE", -6: "RR_ERR_DOMAIN",
                -7: "RR_ERR_NONFINITE", -8: "RR_ERR_CAPACITY"}
GRID_UNIFORM, GRID_OCTREE = 0, 1
FIELD_PHI, FIELD_DELTA, FIELD_PHI_DOT = 0, 1, 2
BOUNDARY_PERIODIC, BOUNDARY_OPEN = 0, 1
PREC_FP64, PREC_FP32_KAHAN = 0, 1
F32, F64 = 0, 1
Q_KAPPA, Q_GAMMA1, Q_GAMMA2, Q_SCALAR = 0, 1, 2, 3
INTEGRAL_TRILINEAR, INTEGRAL_NGP = 0, 1
RAY_OK, RAY_OUT_OF_DOMAIN, RAY_MAX_STEPS, RAY_NONFINITE = 0, 1, 2, 3


class FieldDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("field", C.c_int32), ("boundary", C.c_int32),
                ("dtype", C.c_int32), ("n_base", C.c_int32), ("max_level", C.c_int32),
                ("box_size", C.c_double), ("values", C.c_void_p), ("child_oct", C.c_void_p),
                ("n_cells", C.c_int64)]


class Bundle(C.Structure):
    _fields_ = [("ray_offset", C.c_int64), ("n_rays", C.c_int64), ("dir", C.c_void_p),
                ("nx", C.c_int32), ("ny", C.c_int32), ("chi_s", C.c_double),
                ("chi_hi", C.c_double), ("chi_lo", C.c_double),
                ("center_dir", C.c_double * 3), ("fov_x", C.c_double), ("fov_y", C.c_double)]


class TraceParams(C.Structure):
    _fields_ = [("observer", C.c_double * 3), ("kappa_scale", C.c_double),
                ("precision", C.c_int32), ("quantity", C.c_int32), ("integral", C.c_int32),
                ("persistent", C.c_int32), ("max_crossings", C.c_int64),
                ("crossing_hash", C.c_void_p), ("crossing_count", C.c_void_p),
                ("crossing_log", C.c_void_p), ("log_stride", C.c_int64)]


# (name, restype, argtypes) of every exported entry point
_vp, _i32, _i64 = C.c_void_p, C.c_int32, C.c_int64
SIGNATURES = [
    ("rr_tensor_create", _i32, [C.POINTER(FieldDesc), _i32, C.POINTER(_vp)]),
    ("rr_tensor_destroy", _i32, [_vp]),
    ("rr_build_tidal_tensor", _i32, [_vp, C.POINTER(FieldDesc), _vp]),
    ("rr_build_tidal_tensor_centres", _i32, [_vp, C.POINTER(FieldDesc), _vp]),
    ("rr_build_method_a_fields", _i32, [_vp, C.POINTER(FieldDesc), C.POINTER(FieldDesc),
                                        C.c_double, _vp]),
    ("rr_build_isw_field", _i32, [_vp, C.POINTER(FieldDesc), C.POINTER(FieldDesc), C.c_double,
                                  _vp]),
    ("rr_build_tidal_tensor_box", _i32, [_vp, C.POINTER(FieldDesc), C.POINTER(_i32),
                                         C.POINTER(_i32), _vp]),
    ("rr_tensor_layout", _i32, [_vp, C.POINTER(_vp), C.POINTER(_i64), C.POINTER(_i32),
                                C.POINTER(_i32)]),
    ("rr_plan_create", _i32, [C.POINTER(_vp)]),
    ("rr_plan_destroy", _i32, [_vp]),
    ("rr_trace_rays", _i32, [_vp, _vp, C.POINTER(TraceParams), C.POINTER(Bundle), _i32, _vp, _vp,
                             _vp, _vp]),
    ("rr_trace_rays_noalloc", _i32, [_vp, C.POINTER(TraceParams), C.POINTER(Bundle), _i32, _vp,
                                     _vp, _vp, _vp]),
    ("rr_trace_rays_sources", _i32, [_vp, _vp, C.POINTER(TraceParams), C.POINTER(Bundle), _i32,
                                     C.POINTER(C.c_double), _i32, _vp, _vp, _vp, _vp]),
    ("rr_kappa_from_pieces", _i32, [_vp, _vp, C.POINTER(C.c_double), _i32, _i64, _vp, _vp, _vp,
                                    _vp]),
    ("rr_trace_rays_adjoint", _i32, [_vp, _vp, C.POINTER(FieldDesc), C.POINTER(TraceParams),
                                     C.POINTER(Bundle), _i32, _vp, _vp, _vp]),
    ("rr_rays_vertex_box", _i32, [_vp, _vp, C.POINTER(TraceParams), C.POINTER(Bundle), _i32,
                                  C.POINTER(_i32), C.POINTER(_i32), _vp]),
    ("rr_plan_autotune", _i32, [_vp, _vp, C.POINTER(TraceParams), C.POINTER(Bundle), _i32, _vp]),
    ("rr_plan_set_shape", _i32, [_vp, C.POINTER(Bundle), _i32, _i32, _i32, _i32, _i32]),
    ("rr_plan_tuned_shape", _i32, [_vp, C.POINTER(Bundle), _i32, C.POINTER(_i32), C.POINTER(_i32),
                                   C.POINTER(_i32), C.POINTER(_i32), C.POINTER(C.c_float)]),
    ("rr_graph_begin", _i32, [_vp, _vp]),
    ("rr_graph_end", _i32, [_vp, _vp]),
    ("rr_graph_launch", _i32, [_vp, _vp]),
    ("rr_fov_directions", _i32, [C.POINTER(C.c_double), C.c_double, C.c_double, _i32, _i32,
                                 _vp]),
    ("rr_last_error", C.c_char_p, []),
    ("rr_version", _i32, []),
]

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1601_02012_amd.build` "
                "(hipcc, gfx950).  There is no CPU fallback.")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().rr_last_error().decode()


class RRError(RuntimeError):
    def __init__(self, func: str, status: int, msg: str):
        super().__init__(f"{func} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(func: str, status: int) -> None:
    if status != RR_OK:
        raise RRError(func, status, last_error())
