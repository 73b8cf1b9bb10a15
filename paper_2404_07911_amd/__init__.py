"""MI355X (gfx950) matrix-free unfitted DG operator.

Hot path: v = A u for the SIPG discretisation of the Poisson problem on a
level-set-cut Cartesian mesh (Bergbauer, Munch, Wall, Kronbichler, arXiv
2404.07911), with hand-written HIP kernels behind the C ABI in include/ufem.h.

Every entry point loads libufem.so and raises ImportError if it has not been
built: there is no fallback path.  (`python -m paper_2404_07911_amd.build`
compiles it.)
"""
from . import _lib
from ._lib import (F32, F64, PART_ALL, PART_CUT, PART_CUT_FACE_LINES, PART_CUT_LINES, PART_CUT_STRUCTURED,
                   PART_INSIDE, TERM_ALL, TERM_GHOST, TERM_NITSCHE, TERM_SIPG, TERM_VOLUME, UfemError)
from .ufem import Operator, Plan, Problem, ufem_apply

__all__ = [
    "Plan",
    "Problem",
    "Operator",
    "ufem_apply",
    "UfemError",
    "F64",
    "F32",
    "TERM_ALL",
    "TERM_VOLUME",
    "TERM_SIPG",
    "TERM_NITSCHE",
    "TERM_GHOST",
    "PART_INSIDE",
    "PART_CUT_STRUCTURED",
    "PART_CUT_LINES",
    "PART_CUT_FACE_LINES",
    "PART_CUT",
    "PART_ALL",
]
