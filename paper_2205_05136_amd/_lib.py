"""ctypes binding of libmfsem (include/mfsem.h): structures, prototypes and the
status-to-exception mapping.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MFSEM_LIBRARY may point at another build of the same library (e.g. to compare builds)
LIB_PATH = os.environ.get("MFSEM_LIBRARY") or os.path.join(_HERE, "libmfsem.so")

MFSEM_OK, MFSEM_EINVAL, MFSEM_EUNSUPPORTED, MFSEM_EGEOMETRY = 0, -1, -2, -3
MFSEM_EDEVICE, MFSEM_ENOCONV, MFSEM_EBREAKDOWN, MFSEM_ENONFINITE = -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "EGEOMETRY", -4: "EDEVICE",
                -5: "ENOCONV", -6: "EBREAKDOWN", -7: "ENONFINITE"}
MFSEM_GLL, MFSEM_GAUSS = 0, 1
MFSEM_F64, MFSEM_F32 = 0, 1
MFSEM_TRANSFER_P, MFSEM_TRANSFER_H = 0, 1
MFSEM_GEOM_AUTO, MFSEM_GEOM_STORED, MFSEM_GEOM_ONTHEFLY = 0, 1, 2
MAX_P = 8
NOALLOC_SCRATCH_MB = 64   # MFSEM_NOALLOC_SCRATCH_MB: the fixed scratch of mfsem_pcg_noalloc


class MfsemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"mfsem {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class BoxDesc(C.Structure):
    _fields_ = [("p", C.c_int32), ("n", C.c_int32 * 3), ("origin", C.c_double * 3),
                ("length", C.c_double * 3), ("shear_amp", C.c_double), ("fiber", C.c_int32),
                ("theta0", C.c_double), ("theta1", C.c_double)]


class OpDesc(C.Structure):
    _fields_ = [("p", C.c_int32), ("quad", C.c_int32), ("nq1d", C.c_int32),
                ("n_elem", C.c_int64), ("n_dof", C.c_int64), ("elem_dof", C.c_void_p),
                ("map_p", C.c_int32), ("map_elem_dof", C.c_void_p), ("n_map_nodes", C.c_int64),
                ("map_xyz", C.c_void_p), ("fiber", C.c_void_p), ("sheet", C.c_void_p),
                ("sigma", C.c_void_p), ("sigma_const", C.c_double * 3), ("batch", C.c_int32),
                ("alpha", C.c_double), ("store_f64", C.c_int32), ("store_f32", C.c_int32),
                ("lattice", C.c_int32 * 3), ("geometry", C.c_int32)]


class TransferDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("parent", C.c_void_p), ("child", C.c_void_p)]


class MgDesc(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("ops", C.POINTER(C.c_void_p)),
                ("transfers", C.POINTER(TransferDesc)), ("degree", C.c_int32),
                ("coarse_degree", C.c_int32), ("lo_frac", C.c_double), ("hi_frac", C.c_double),
                ("eig_iters", C.c_int32), ("eig_seed", C.c_uint64),
                ("lambda_max", C.POINTER(C.c_double)), ("precision", C.c_int32),
                ("graphs", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_it", C.c_int32),
                ("flexible", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("r0_norm", C.c_double),
                ("r_norm", C.c_double), ("b_norm", C.c_double)]


class APParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("k", "a", "eps0", "mu1", "mu2", "v_rest", "v_amp",
                                          "t_scale")]


_P = C.c_void_p
_ST = C.c_int
PROTOTYPES = {
    "mfsem_abi_version": (C.c_int, []),
    "mfsem_last_error": (C.c_char_p, []),
    "mfsem_box_counts": (_ST, [C.POINTER(BoxDesc), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mfsem_box_generate": (_ST, [C.POINTER(BoxDesc), _P, _P, _P, _P]),
    "mfsem_box_parents": (_ST, [C.POINTER(C.c_int32), _P, _P, _P]),
    "mfsem_mesh_refine_nodes": (_ST, [C.c_int32, C.c_int64, _P, C.c_int64, _P, _P, C.c_int64, _P,
                                      _P, _P, _P, _P]),
    "mfsem_mesh_degree_nodes": (_ST, [C.c_int32, C.c_int64, _P, C.c_int64, _P, _P, C.c_int32,
                                      C.c_int64, _P, _P, _P, _P, _P]),
    "mfsem_op_workspace_bytes": (_ST, [C.POINTER(OpDesc), C.POINTER(C.c_size_t)]),
    "mfsem_op_create": (_ST, [C.POINTER(OpDesc), _P, C.c_size_t, _P, C.POINTER(_P)]),
    "mfsem_op_destroy": (_ST, [_P]),
    "mfsem_op_set_alpha": (_ST, [_P, C.c_double]),
    "mfsem_op_set_sigma": (_ST, [_P, _P, _P]),
    "mfsem_op_apply": (_ST, [_P, C.c_int32, _P, _P, _P]),
    "mfsem_op_apply_add": (_ST, [_P, C.c_int32, _P, _P, _P]),
    "mfsem_op_apply_mass": (_ST, [_P, C.c_int32, _P, _P, _P]),
    "mfsem_op_diagonal": (_ST, [_P, C.c_int32, _P, _P]),
    "mfsem_op_grad_sigma": (_ST, [_P, _P, _P, C.c_double, _P, _P]),
    "mfsem_csr_nnz": (_ST, [_P, C.c_int, C.POINTER(C.c_int64)]),
    "mfsem_csr_assemble": (_ST, [_P, C.c_int, _P, _P, _P, _P]),
    "mfsem_csr_spmv": (_ST, [C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P]),
    "mfsem_extrapolate": (_ST, [C.c_int64, _P, _P, _P, _P]),
    "mfsem_mg_workspace_bytes": (_ST, [C.POINTER(MgDesc), C.POINTER(C.c_size_t)]),
    "mfsem_mg_create": (_ST, [C.POINTER(MgDesc), _P, C.c_size_t, _P, C.POINTER(_P)]),
    "mfsem_mg_destroy": (_ST, [_P]),
    "mfsem_mg_vcycle": (_ST, [_P, _P, _P, _P]),
    "mfsem_mg_lambdas": (_ST, [_P, C.POINTER(C.c_double)]),
    "mfsem_mg_transfer": (_ST, [_P, C.c_int32, C.c_int32, _P, _P, _P]),
    "mfsem_pcg_workspace_bytes": (_ST, [_P, _P, C.POINTER(C.c_size_t)]),
    "mfsem_pcg": (_ST, [_P, _P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P,
                        C.c_size_t, _P]),
    "mfsem_pcg_noalloc": (_ST, [_P, _P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "mfsem_ap_imex_rhs": (_ST, [C.c_int64, C.c_double, C.c_double, C.c_double,
                                C.POINTER(APParams), _P, _P, _P, _P, _P, _P]),
    "mfsem_ap_bdf2_rhs": (_ST, [C.c_int64, C.c_double, C.c_double, C.c_double,
                                C.POINTER(APParams), _P, _P, _P, _P, _P, _P, _P, _P]),
    "mfsem_activation_update": (_ST, [C.c_int64, C.c_double, C.c_double, _P, _P, _P, _P,
                                      C.c_double, _P, _P]),
}

_lib = None


def load():
    """Load the in-tree libmfsem.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2205_05136_amd.build` (there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != MFSEM_OK:
        msg = load().mfsem_last_error().decode(errors="replace")
        raise MfsemError(status, msg)
