"""mfsem: matrix-free spectral-element monodomain operator and GMG-PCG for
AMD Instinct MI355X (gfx950).

The compute path is the HIP library libmfsem.so (C ABI in include/mfsem.h);
this package is its Python binding.  Importing it does not load the library;
the first call does, and fails loudly if the library was not built.
"""
from . import _lib
from ._lib import MfsemError
from .api import (Box, CsrMatrix, Multigrid, Operator, SolveInfo, abi_version, ap_bdf2_rhs,
                  activation_update, ap_imex_rhs, box_parents, extrapolate, hierarchy, pcg)

__all__ = ["Box", "Operator", "CsrMatrix", "Multigrid", "SolveInfo", "MfsemError", "abi_version",
           "pcg", "hierarchy", "box_parents", "ap_imex_rhs", "ap_bdf2_rhs", "activation_update",
           "extrapolate"]
