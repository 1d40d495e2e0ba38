"""ctypes loader for libtetct.so: the C interface of include/tetct.h, same names.

Argument marshalling only.  Loading fails loudly when the library has not
been built; there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TCT_LIB_PATH selects another build of the same library (the sanitizer
# tests load an instrumented one); by default the in-tree build.
LIB_PATH = os.environ.get("TCT_LIB_PATH") or os.path.join(HERE, "libtetct.so")

STATUS = {
    0: "TCT_OK",
    -1: "TCT_E_ARG",
    -2: "TCT_E_MESH_DEGENERATE",
    -3: "TCT_E_MESH_NONMANIFOLD",
    -4: "TCT_E_MESH_NONCONVEX",
    -5: "TCT_E_MESH_DISCONNECTED",
    -6: "TCT_E_GEOM",
    -7: "TCT_E_NOMEM",
    -8: "TCT_E_HIP",
    -9: "TCT_E_WALK",
    -10: "TCT_E_CAPACITY",
}

TCT_MESH_NO_REORDER = 1
TCT_MESH_HOST_ONLY = 2
TCT_MESH_RSTAR = 4
TCT_BP_ATOMIC = 0
TCT_BP_GATHER = 1
TCT_BP_ATOMIC_DIRECT = 2
TCT_BP_SHADOW = 3
TCT_BP_FIXED = 4
TCT_NOALLOC_MAX_TETS = 4194304
TCT_DOT_WORKSPACE = 512
TCT_VECSET_DOT_WORKSPACE = 256


class TctError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class tct_cone(C.Structure):
    _fields_ = [("dso", C.c_double), ("dsd", C.c_double), ("nu", C.c_int32), ("nv", C.c_int32),
                ("du", C.c_double), ("dv", C.c_double), ("off_u", C.c_double), ("off_v", C.c_double)]


class tct_range(C.Structure):
    _fields_ = [("a0", C.c_int32), ("na", C.c_int32), ("tile_u", C.c_int32)]


class tct_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in
                ("rays", "segments", "zero_len", "fp64_stage", "exact_stage", "perturbed_ties", "failed", "grazing_fp64")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class tct_paper_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("rays", "steps", "escalations", "halted", "looped")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


# name -> (restype, argtypes); pointers are passed as integers (c_void_p).
_P = C.c_void_p
_SIGS = {
    "tct_mesh_create": (C.c_int, [_P, C.c_int32, _P, C.c_int32, _P, C.c_uint32, C.c_int, C.POINTER(_P)]),
    "tct_mesh_counts": (C.c_int, [_P, _P, _P, _P, _P]),
    "tct_mesh_permutation": (C.c_int, [_P, _P]),
    "tct_mesh_boundary": (C.c_int, [_P, _P, _P]),
    "tct_mesh_rstar": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "tct_mesh_neighbors": (C.c_int, [_P, _P]),
    "tct_mesh_to_internal": (C.c_int, [_P, _P, _P, _P]),
    "tct_mesh_to_user": (C.c_int, [_P, _P, _P, _P]),
    "tct_stats_read": (C.c_int, [_P, C.POINTER(tct_stats), C.c_int]),
    "tct_mesh_destroy": (None, [_P]),
    "tct_geom_create": (C.c_int, [C.POINTER(tct_cone), _P, C.c_int32, C.c_int, C.POINTER(_P)]),
    "tct_geom_nrays": (C.c_int64, [_P]),
    "tct_geom_frame": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "tct_geom_destroy": (None, [_P]),
    "tct_entry": (C.c_int, [_P, _P, _P, _P]),
    "tct_entry_rstar": (C.c_int, [_P, _P, _P, _P]),
    "tct_entry_raster": (C.c_int, [_P, _P, _P, _P]),
    "tct_forward": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "tct_backproject": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, _P, _P]),
    "tct_trace": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P, C.c_int64, C.POINTER(C.c_int64), _P]),
    "tct_trace_rays": (C.c_int, [_P, _P, _P, _P, _P, C.c_int32, _P, _P, _P, C.c_int64, C.POINTER(C.c_int64), _P]),
    "tct_dot": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P]),
    "tct_axpy_ratio": (C.c_int, [_P, _P, C.c_int64, _P, _P, C.c_double, _P]),
    "tct_xpay_ratio": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P]),
    "tct_axpby": (C.c_int, [_P, _P, C.c_int64, C.c_float, C.c_float, _P]),
    "tct_mul": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "tct_recip": (C.c_int, [_P, _P, C.c_int64, C.c_float, _P]),
    "tct_copy_f64": (C.c_int, [_P, _P, C.c_int32, _P]),
    "tct_forward_range": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "tct_forward_paper": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.POINTER(tct_paper_stats), _P]),
    "tct_backproject_range": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, _P, _P, _P]),
    "tct_backproject_fixed_noalloc": (C.c_int, [_P, _P, _P, _P, C.c_int, _P, _P]),
    "tct_vecset_create": (C.c_int, [C.c_int32, _P, _P, C.c_int, C.POINTER(_P)]),
    "tct_vecset_destroy": (None, [_P]),
    "tct_vecset_dot": (C.c_int, [_P, _P, _P, _P, _P]),
    "tct_vecset_axpy_ratio": (C.c_int, [_P, _P, _P, _P, C.c_double, _P]),
    "tct_vecset_xpay_ratio": (C.c_int, [_P, _P, _P, _P, _P]),
    "tct_vecset_fill": (C.c_int, [_P, C.c_float, _P]),
    "tct_batch_create": (C.c_int, [_P, _P, C.c_int32, _P, _P, C.POINTER(_P)]),
    "tct_batch_forward": (C.c_int, [_P, _P, _P, _P]),
    "tct_batch_backproject": (C.c_int, [_P, _P, _P, C.c_int, _P]),
    "tct_batch_items": (C.c_int64, [_P]),
    "tct_batch_set_queue_chunk": (C.c_int, [_P, C.c_int32]),
    "tct_batch_destroy": (None, [_P]),
    "tct_last_error": (C.c_char_p, []),
    "tct_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library; raises if libtetct.so is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1908_06909_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def check(status: int):
    if status != 0:
        raise TctError(status, lib().tct_last_error().decode(errors="replace"))
    return status


def call(name, *args):
    return check(getattr(lib(), name)(*args))
