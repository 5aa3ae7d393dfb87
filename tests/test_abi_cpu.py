"""The C-ABI library loads on the CPU, exports every symbol its header
declares, agrees with the header on structure layouts, and validates
arguments on the host (no device calls)."""
import ctypes as C
import os
import re
import subprocess

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfsem.h")

mf = pytest.importorskip("paper_2205_05136_amd")
L = mf._lib


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mfsem_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a prototype for each
    assert set(names) <= set(L.PROTOTYPES), set(names) - set(L.PROTOTYPES)
    hdr = open(os.path.join(ROOT, "include", "mfsem.h")).read()
    assert f"#define MFSEM_ABI_VERSION {lib.mfsem_abi_version()}\n" in hdr


def test_struct_layouts_match_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mfsem.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                    'sizeof(mfsem_box_desc), sizeof(mfsem_op_desc), sizeof(mfsem_mg_desc),'
                    'sizeof(mfsem_transfer_desc), sizeof(mfsem_solve_opts), sizeof(mfsem_solve_info),'
                    'sizeof(mfsem_ap_params), offsetof(mfsem_op_desc, alpha),'
                    'offsetof(mfsem_op_desc, geometry), offsetof(mfsem_mg_desc, graphs));'
                    'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(L.BoxDesc), C.sizeof(L.OpDesc), C.sizeof(L.MgDesc),
            C.sizeof(L.TransferDesc), C.sizeof(L.SolveOpts), C.sizeof(L.SolveInfo),
            C.sizeof(L.APParams), L.OpDesc.alpha.offset, L.OpDesc.geometry.offset,
            L.MgDesc.graphs.offset]
    assert got == want


def _box(p=4, n=(40, 14, 6)):
    return L.BoxDesc(p=p, n=(C.c_int32 * 3)(*n), length=(C.c_double * 3)(20, 7, 3))


def test_box_counts_and_validation():
    lib = L.load()
    ne, nd = C.c_int64(), C.c_int64()
    assert lib.mfsem_box_counts(C.byref(_box()), C.byref(ne), C.byref(nd)) == 0
    assert (ne.value, nd.value) == (synth.C2.n_elem, synth.C2.n_dof)
    assert lib.mfsem_box_counts(C.byref(_box(p=9)), C.byref(ne), C.byref(nd)) == L.MFSEM_EINVAL
    assert b"MFSEM_MAX_P" in lib.mfsem_last_error()
    assert lib.mfsem_box_counts(C.byref(_box(n=(0, 1, 1))), C.byref(ne), C.byref(nd)) == -1
    assert lib.mfsem_box_counts(None, C.byref(ne), C.byref(nd)) == -1


def _op_desc(**kw):
    d = L.OpDesc(p=4, quad=L.MFSEM_GLL, nq1d=0, n_elem=10, n_dof=100, elem_dof=1, map_p=0,
                 map_elem_dof=None, n_map_nodes=100, map_xyz=1, fiber=None, sheet=None,
                 sigma=None, sigma_const=(C.c_double * 3)(1, 1, 1), batch=1, alpha=1.0,
                 store_f64=1, store_f32=0)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_op_workspace_query_and_validation():
    lib = L.load()
    nb = C.c_size_t()
    assert lib.mfsem_op_workspace_bytes(C.byref(_op_desc()), C.byref(nb)) == 0
    # G (6) + WJ (1) doubles per point, 125 points, 10 elements, plus tables
    assert nb.value >= 10 * 125 * 7 * 8
    nb32 = C.c_size_t()
    lib.mfsem_op_workspace_bytes(C.byref(_op_desc(store_f64=0, store_f32=1)), C.byref(nb32))
    assert nb32.value < nb.value
    bad = [dict(p=0), dict(p=9), dict(quad=5), dict(nq1d=7), dict(quad=L.MFSEM_GAUSS, nq1d=4),
           dict(quad=L.MFSEM_GAUSS, nq1d=9), dict(batch=0), dict(alpha=-1.0),
           dict(store_f64=0, store_f32=0), dict(map_p=3), dict(elem_dof=None),
           dict(sheet=5), dict(n_dof=2 ** 31), dict(geometry=3), dict(geometry=-1),
           # on-the-fly geometry needs a structured GLL lattice whose map is the DOF nodes
           dict(geometry=L.MFSEM_GEOM_ONTHEFLY)]
    for kw in bad:
        assert lib.mfsem_op_workspace_bytes(C.byref(_op_desc(**kw)), C.byref(nb)) == -1, kw
        assert lib.mfsem_last_error()
    assert lib.mfsem_op_workspace_bytes(C.byref(_op_desc(quad=L.MFSEM_GAUSS, nq1d=7)),
                                        C.byref(nb)) == 0


def test_null_handles_are_rejected_without_a_device():
    lib = L.load()
    assert lib.mfsem_op_destroy(None) == 0
    assert lib.mfsem_mg_destroy(None) == 0
    assert lib.mfsem_op_apply(None, 0, None, None, None) == -1
    assert lib.mfsem_op_set_alpha(None, 1.0) == -1
    assert lib.mfsem_mg_vcycle(None, None, None, None) == -1
    info = (L.SolveInfo * 1)()
    opts = L.SolveOpts(rtol=1e-10, atol=0, max_it=10, flexible=0)
    assert lib.mfsem_pcg(None, None, None, None, C.byref(opts), info, None, 0, None) == -1
    prm = L.APParams(k=8, a=0.15, eps0=0.002, mu1=0.2, mu2=0.3, v_rest=-80, v_amp=100, t_scale=0)
    assert lib.mfsem_ap_imex_rhs(0, 0.05, 140, 0.01, C.byref(prm), None, None, None, None, None,
                                 None) == -1
    n = (C.c_int32 * 3)(3, 2, 2)
    assert lib.mfsem_box_parents(n, None, None, None) == -1
    nnz = C.c_int64()
    assert lib.mfsem_csr_nnz(None, 0, C.byref(nnz)) == -1
    assert lib.mfsem_csr_spmv(-1, 0, None, None, None, None, None, None) == -1
    assert lib.mfsem_extrapolate(-1, None, None, None, None) == -1
    assert lib.mfsem_extrapolate(5, None, None, None, None) == -1
    assert lib.mfsem_extrapolate(0, None, None, None, None) == 0
    assert lib.mfsem_csr_spmv(4, -1, None, None, None, None, None, None) == -1
