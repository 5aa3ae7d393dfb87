"""mfsem_pcg_noalloc (the PCG entry point that allocates nothing: its work
vectors live in the library's fixed per-device scratch array) called through
the C ABI, against mfsem_pcg with a caller workspace: the same solutions to
the FP64 bar, on two calls in a row, the second on a smaller problem (the
scratch keeps the first call's contents), and a clear EINVAL for a problem
beyond the scratch, before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_common import announce, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

mf = pytest.importorskip("paper_2205_05136_amd")
L = mf._lib
from paper_2205_05136_amd import api  # noqa: E402


def _pcg_noalloc(op, b, mg=None, rtol=1e-13, max_it=500, flexible=False):
    lib = L.load()
    x = torch.zeros_like(b)
    opts = L.SolveOpts(rtol=rtol, atol=0.0, max_it=max_it, flexible=int(flexible))
    infos = (L.SolveInfo * op.batch)()
    st = lib.mfsem_pcg_noalloc(op.handle, mg.handle if mg else None, api._ptr(b), api._ptr(x),
                               C.byref(opts), infos, api._stream())
    return st, x, [i.iters for i in infos], [i.status for i in infos]


def test_pcg_noalloc_matches_pcg_twice_then_smaller():
    announce("pcg noalloc: two calls, the second smaller")
    big = synth.slab(4, (12, 6, 4))
    small = synth.slab(3, (5, 4, 3))
    # first call: GMG-PCG (FP64 V-cycle); second: a smaller plain CG in the same scratch
    ops, mg = mf.hierarchy(big, coarsening=(("p", 2), ("p", 1)), degree=3)
    f1 = to_dev(synth.uniform(21, big.n_dof))
    st, x1, it1, s1 = _pcg_noalloc(ops[0], f1, mg=mg)
    assert st == 0 and s1 == [0], L.load().mfsem_last_error()
    ref1, info1 = mf.pcg(ops[0], f1, mg=mg, rtol=1e-13, max_it=500)
    assert rel_l2(to_np(x1), to_np(ref1)) <= 1e-12 and it1 == info1.iters
    op2 = mf.Operator.from_spec(small)
    f2 = to_dev(synth.uniform(22, small.n_dof))
    st, x2, it2, s2 = _pcg_noalloc(op2, f2)
    assert st == 0 and s2 == [0], L.load().mfsem_last_error()
    ref2, info2 = mf.pcg(op2, f2, rtol=1e-13, max_it=500)
    assert rel_l2(to_np(x2), to_np(ref2)) <= 1e-12
    # the mixed-precision solve (FP32 V-cycle, flexible CG) uses the FP32 vectors of the scratch too
    ops32, mg32 = mf.hierarchy(big, coarsening=(("p", 2), ("p", 1)), degree=3,
                               precision=torch.float32)
    st, x3, _, _ = _pcg_noalloc(ops32[0], f1, mg=mg32, rtol=1e-10, flexible=True)
    ref3, _ = mf.pcg(ops32[0], f1, mg=mg32, rtol=1e-10, max_it=500)
    assert st == 0 and rel_l2(to_np(x3), to_np(ref3)) <= 1e-12
    assert rel_l2(to_np(x3), to_np(ref1)) <= 1e-8


def test_pcg_noalloc_rejects_problems_beyond_the_scratch():
    announce("pcg noalloc: too large")
    spec = synth.BoxSpec(p=2, n=(64, 64, 64))          # 2,146,689 DOFs: ~86 MB of CG vectors
    op = mf.Operator.from_spec(spec)
    nbytes = C.c_size_t()
    L.check(L.load().mfsem_pcg_workspace_bytes(op.handle, None, C.byref(nbytes)))
    assert nbytes.value > (L.NOALLOC_SCRATCH_MB << 20)
    f = torch.ones(spec.n_dof, dtype=torch.float64, device="cuda")
    st, x, _, _ = _pcg_noalloc(op, f, max_it=3)
    assert st == L.MFSEM_EINVAL
    assert "scratch" in L.load().mfsem_last_error().decode()
    assert float(x.abs().max()) == 0.0   # nothing was launched
