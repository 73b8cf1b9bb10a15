"""ctypes binding of libufem.so (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libufem.so")

UFEM_OK, UFEM_EINVAL, UFEM_ENOMEM, UFEM_EHIP, UFEM_EUNSUPPORTED, UFEM_ESTATE = 0, -1, -2, -3, -4, -5
TERM_VOLUME, TERM_SIPG, TERM_NITSCHE, TERM_GHOST, TERM_ALL = 1, 2, 4, 8, 15
F64, F32 = 0, 1
LEVELSET_BALLS, LEVELSET_PLANE = 0, 1
GP_FACE, GP_VOLUME, GP_VOLUME_ALL = 0, 1, 2
SPACE_DG, SPACE_CG = 0, 1
PART_INSIDE, PART_CUT_STRUCTURED, PART_CUT_LINES, PART_CUT_FACE_LINES = 1, 2, 4, 8
PART_CUT, PART_ALL = 14, 15


class ufem_problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("n", C.c_int32),
        ("lo", C.c_double),
        ("hi", C.c_double),
        ("degree", C.c_int32),
        ("q_cut", C.c_int32),
        ("max_depth", C.c_int32),
        ("n_balls", C.c_int32),
        ("centers", C.POINTER(C.c_double)),
        ("radii", C.POINTER(C.c_double)),
        ("nitsche_factor", C.c_double),
        ("sipg_factor", C.c_double),
        ("gp_gamma", C.c_double),
        ("gp_jmin", C.c_int32),
        ("gp_flat", C.c_int32),
        ("levelset", C.c_int32),
        ("plane_normal", C.c_double * 3),
        ("plane_offset", C.c_double),
        ("gp_kind", C.c_int32),
        ("space", C.c_int32),
    ]


class ufem_info(C.Structure):
    _fields_ = [
        ("n_background", C.c_int64),
        ("n_active", C.c_int64),
        ("n_inside", C.c_int64),
        ("n_cut", C.c_int64),
        ("n_dofs", C.c_int64),
        ("n_faces", C.c_int64),
        ("n_faces_str", C.c_int64),
        ("n_faces_cut", C.c_int64),
        ("n_faces_gp", C.c_int64),
        ("n_qp", C.c_int64),
        ("seg", C.c_int64 * 6),
        ("max_qp_cut_cell", C.c_int64),
        ("n_fallback", C.c_int64),
        ("h", C.c_double),
        ("n_cell_dofs", C.c_int64),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "seg"}
        d["seg"] = list(self.seg)
        return d


class UfemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ufem error {code}: {msg}")
        self.code = code


_vp = C.c_void_p
_SIGS = {
    "ufem_last_error": (C.c_char_p, []),
    "ufem_plan_create": (C.c_int, [C.POINTER(ufem_problem), C.POINTER(_vp)]),
    "ufem_plan_destroy": (C.c_int, [_vp]),
    "ufem_plan_info": (C.c_int, [_vp, C.POINTER(ufem_info)]),
    "ufem_plan_cells": (C.c_int, [_vp, _vp]),
    "ufem_plan_faces": (C.c_int, [_vp, _vp]),
    "ufem_plan_qp": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ufem_plan_import_quadrature": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ufem_setup": (C.c_int, [_vp, C.c_int, _vp, C.c_int64, C.POINTER(_vp)]),
    "ufem_destroy": (C.c_int, [_vp]),
    "ufem_info_op": (C.c_int, [_vp, C.POINTER(ufem_info)]),
    "ufem_set_terms": (C.c_int, [_vp, C.c_int32]),
    "ufem_set_max_blocks": (C.c_int, [_vp, C.c_int32]),
    "ufem_set_mixed": (C.c_int, [_vp, C.c_int32, _vp]),
    "ufem_set_kappa": (C.c_int, [_vp, C.c_int32, _vp, _vp]),
    "ufem_apply": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp]),
    "ufem_apply_part": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp]),
    "ufem_apply_adjoint": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "ufem_cg_iterate": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ufem_cg_iterate_static": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "ufem_dot": (C.c_int, [C.c_int32, C.c_int64, _vp, _vp, _vp, _vp]),
    "ufem_axpby": (C.c_int, [C.c_int32, C.c_int64, C.c_double, _vp, C.c_double, _vp, _vp]),
    "ufem_cast": (C.c_int, [C.c_int32, C.c_int32, C.c_int64, _vp, _vp, _vp]),
}

_lib = None


def lib():
    """Load libufem.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2404_07911_amd.build` "
                "(or __graft_entry__.build())"
            )
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != UFEM_OK:
        msg = lib().ufem_last_error().decode(errors="replace")
        raise UfemError(code, msg)
    return code


def exported_symbols():
    return list(_SIGS)
