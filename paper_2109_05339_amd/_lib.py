"""ctypes loader of libspfel.so and its status codes.

The library is built in-tree (``python -m paper_2109_05339_amd.build``);
importing the package without it raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspfel.so")

OK, EINVAL, ERANGE, ENOMEM, EHIP, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6


class SpfelError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"spfel error {code}: {msg}")
        self.code = code


class SpfelInvalidArgument(SpfelError, ValueError):
    pass


class SpfelStateError(SpfelError):
    pass


class SpfelUnsupported(SpfelError, NotImplementedError):
    pass


class SpfelOutOfMemory(SpfelError, MemoryError):
    pass


_ERRORS = {EINVAL: SpfelInvalidArgument, ERANGE: SpfelInvalidArgument, ESTATE: SpfelStateError,
           EUNSUPPORTED: SpfelUnsupported, ENOMEM: SpfelOutOfMemory}

_vp, _i64, _int, _dbl, _flt, _sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_float, ctypes.c_size_t)

# name -> (restype, argtypes); the same list the header declares.
SIGNATURES = {
    "spfel_version": (_int, []),
    "spfel_last_error": (ctypes.c_char_p, []),
    "spfel_plan_create": (_int, [ctypes.POINTER(_vp), _int, _int, _dbl, _dbl, _int, _int]),
    "spfel_plan_destroy": (_int, [_vp]),
    "spfel_plan_info": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_sz)]),
    "spfel_set_detector": (_int, [_vp, _vp, _i64, _vp]),
    "spfel_set_model": (_int, [_vp, _vp, _vp]),
    "spfel_slice": (_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp]),
    "spfel_row_norm2": (_int, [_vp, _int, _i64, _i64, _vp, _vp]),
    "spfel_column_mean": (_int, [_vp, _i64, _i64, _int, _vp, _vp]),
    "spfel_bf16_centred": (_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp]),
    "spfel_match_workspace_bytes": (_sz, [_i64, _i64, _i64, _int]),
    "spfel_match": (_int, [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _int, _vp, _vp, _vp, _vp,
                           _vp, _vp, _vp, _vp, _sz, _vp]),
    "spfel_match_noalloc": (_int, [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _int, _vp, _vp,
                                   _vp, _vp, _vp, _vp, _vp, _vp]),
    "spfel_orient_workspace_bytes": (_sz, [_i64, _i64, _i64, _int]),
    "spfel_orient": (_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _int,
                            _i64, _vp, _vp, _vp, _vp, _sz, _vp, _vp]),
    "spfel_scale_columns": (_int, [_vp, _i64, _i64, _vp, _vp, _vp]),
    "spfel_merge_adjoint": (_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _int, _vp]),
    "spfel_weighted_residual": (_int, [_vp, _vp, _vp, _vp, _i64, _flt, _vp, _vp, _vp, _vp]),
    "spfel_normal_create": (_int, [ctypes.POINTER(_vp), _int, _int, _int, _int]),
    "spfel_normal_destroy": (_int, [_vp]),
    "spfel_normal_set_psf": (_int, [_vp, _vp, _vp]),
    "spfel_normal_apply": (_int, [_vp, _vp, _int, _vp, _vp, _vp]),
    "spfel_normal_solve": (_int, [_vp, _vp, _vp, _int, _vp, _int, _vp, _vp, _vp]),
    "spfel_normal_lcurve": (_int, [_vp, _vp, _vp, _vp, _int, _vp, _dbl, _vp, _vp, _vp]),
    "spfel_phase_create": (_int, [ctypes.POINTER(_vp), _int, _int]),
    "spfel_phase_destroy": (_int, [_vp]),
    "spfel_phase_iterate": (_int, [_vp, _vp, _vp, _vp, _vp, _int, _int, _flt, _int, _vp, _vp]),
    "spfel_phase_shrinkwrap": (_int, [_vp, _vp, _flt, _flt, _vp, _vp, _vp]),
}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2109_05339_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(code: int) -> None:
    if code != OK:
        msg = lib().spfel_last_error().decode(errors="replace")
        raise _ERRORS.get(code, SpfelError)(code, msg)
