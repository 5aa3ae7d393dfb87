"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: FP64 relative L2 <= 1e-12 (apply, mass, diagonal, transfers, V-cycle,
solve, gradient); integer outputs bit-exact; FP32 applies <= 1e-5 (rounding of
G and vectors to single precision: ~P^4 terms of size 1 summed per output,
each with relative error 6e-8); mixed-precision solves <= 1e-8 against the
FP64 solution."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import synth
from gpu_common import announce, jitter_scale, oracle_problem, rel_l2, to_dev, to_np
from oracle import adjoint as oadj
from oracle import ionic as oion
from oracle import mesh as omesh
from oracle import multigrid as omg
from oracle import operator as oop
from oracle import solvers as osol

pytestmark = pytest.mark.gpu

mf = pytest.importorskip("paper_2205_05136_amd")

TOL64 = 1e-12
TOL32 = 1e-5

# Meshes that span several workgroups and leave a ragged last one (p <= 5:
# 63 elements; p >= 6: 10 elements, which the oracle still assembles in seconds).
RAG = (7, 3, 3)
RAG_HI = (5, 2, 1)


def _spec(p, n=None, **kw):
    n = n or (RAG if p <= 5 else RAG_HI)
    return synth.slab(p, n).with_(**kw)


def _op(spec, jitter=None, sigma=None, **kw):
    box = mf.Box.from_spec(spec)
    xyz = None
    if jitter is not None:
        xyz = box.xyz + to_dev(synth.node_jitter(jitter[0], spec.n_dof, jitter[1]))
    return mf.Operator.from_spec(spec, box=box, xyz=xyz, sigma=sigma, **kw), box


# ------------------------------------------------------------------ meshes ---
@pytest.mark.parametrize("spec", [synth.C1, _spec(4), _spec(7, (3, 2, 2)), synth.C2],
                         ids=["c1", "slab-p4", "slab-p7", "c2"])
def test_box_matches_oracle(spec):
    announce(f"box {spec.p} {spec.n}")
    box = mf.Box.from_spec(spec)
    m = omesh.box(spec)
    assert np.array_equal(box.elem_dof.cpu().numpy().astype(np.int64), m.elem_dof)
    np.testing.assert_allclose(to_np(box.xyz), m.xyz, rtol=0, atol=1e-13 * max(spec.length))
    if spec.fiber:
        np.testing.assert_allclose(to_np(box.fiber), m.fiber, rtol=0, atol=1e-14)


# ------------------------------------------------------------------- apply ---
APPLY_CASES = (
    [("c1", synth.C1, None, None)]
    + [(f"gll-p{p}", _spec(p), None, None) for p in range(1, 9)]
    + [("gll-p3-jitter", _spec(3), (17, None), None),
       ("gll-p5-sigma", _spec(5), None, 3),
       ("gll-p2-iso-jitter", synth.BoxSpec(p=2, n=(5, 4, 3), length=(1.0, 0.8, 0.6),
                                           sigma=(0.3, 0.3, 0.3), alpha=2.5), (5, None), None)]
    + [(f"gauss-p{p}-q{q}", _spec(p, quad="gauss", nq1d=q), None, None)
       for p, q in [(1, 2), (2, 3), (2, 4), (3, 6), (4, 5), (4, 6), (5, 7), (6, 7), (6, 8), (7, 9),
                    (8, 11)]]
    + [("gauss-p3-jitter-sigma", _spec(3, quad="gauss", nq1d=5), (23, None), 8)]
)


@pytest.mark.parametrize("name,spec,jit,sseed", APPLY_CASES, ids=[c[0] for c in APPLY_CASES])
def test_apply_f64(name, spec, jit, sseed):
    announce(f"apply f64 {name}")
    if jit is not None:
        jit = (jit[0], jitter_scale(spec))
    prob, A, M, K = oracle_problem(spec, sigma_seed=sseed, jitter=jit)
    sigma = None if sseed is None else to_dev(prob.sigma)
    op, _ = _op(spec, jitter=jit, sigma=sigma)
    x = synth.uniform(100, spec.n_dof)
    y = to_np(op.apply(to_dev(x)))
    assert rel_l2(y, A @ x) <= TOL64
    if spec.quad == "gll":
        # GLL lattices take the lattice kernel on stored G by default; the same
        # kernel with on-the-fly geometry (p <= 6), and the general element-map
        # kernel, must agree with the oracle too
        variants = [dict(structured=False)] + ([dict(geom="onthefly")] if spec.p <= 6 else [])
        for kw in variants:
            opv, _ = _op(spec, jitter=jit, sigma=sigma, **kw)
            assert rel_l2(to_np(opv.apply(to_dev(x))), A @ x) <= TOL64, kw
    ym = to_np(op.apply_mass(to_dev(x)))
    assert rel_l2(ym, M @ x) <= TOL64
    d = to_np(op.diagonal())
    assert rel_l2(d, A.diagonal()) <= TOL64


# Structured meshes of hundreds of lattice-kernel bricks (more than a workgroup
# per CU), each with ragged bricks on every axis the brick shape splits: sampled
# rows against the oracle's element matrices, and the whole vector against the
# general element kernel (itself pinned above).
BRICK_CASES = [(1, (67, 33, 17)), (2, (41, 29, 9)), (3, (35, 6, 5)), (4, (21, 17, 15)),
               (5, (13, 7, 5)), (6, (17, 15, 9)), (7, (5, 3, 5))]


@pytest.mark.parametrize("p,n", BRICK_CASES, ids=[f"p{c[0]}" for c in BRICK_CASES])
def test_apply_large_bricks(p, n):
    announce(f"apply large bricks p{p} {n}")
    spec = synth.slab(p, n)
    box = mf.Box.from_spec(spec)
    x = torch.sin(0.37 * torch.arange(spec.n_dof, device="cuda", dtype=torch.float64))
    for store32 in (False, True):
        lattice = mf.Operator.from_spec(spec, box=box, store_f32=store32)
        general = mf.Operator.from_spec(spec, box=box, store_f32=store32, structured=False)
        xs = x if not store32 else x.float()
        y, yg = lattice.apply(xs), general.apply(xs)
        assert rel_l2(to_np(y), to_np(yg)) <= (TOL64 if not store32 else TOL32)
        if not store32 and p <= 6:  # the lattice kernel with on-the-fly geometry as well
            otf = mf.Operator.from_spec(spec, box=box, geom="onthefly")
            assert rel_l2(to_np(otf.apply(xs)), to_np(yg)) <= TOL64
        if not store32:
            rng = np.random.default_rng(p)
            rows = np.concatenate([rng.integers(0, spec.n_dof, 24), [0, spec.n_dof - 1]])
            ref = oop.apply_rows(spec, lambda g: np.sin(0.37 * np.asarray(g, dtype=np.float64)),
                                 rows)
            got = to_np(y[torch.as_tensor(rows, device="cuda")])
            assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(ref).max()


# Degenerate shapes: a single element, and meshes one element thick in two
# directions (every brick ragged), at every degree.
EDGE_CASES = [(p, n) for p in (1, 2, 4, 5, 7, 8) for n in ((1, 1, 1), (9, 1, 1), (1, 5, 3))]


@pytest.mark.parametrize("p,n", EDGE_CASES, ids=[f"p{c[0]}-{c[1][0]}x{c[1][1]}x{c[1][2]}"
                                                   for c in EDGE_CASES])
def test_apply_degenerate_meshes(p, n):
    announce(f"apply degenerate p{p} {n}")
    spec = synth.slab(p, n)
    prob, A, M, K = oracle_problem(spec)
    x = synth.uniform(105, spec.n_dof)
    for kw in (dict(), dict(structured=False)):
        op, _ = _op(spec, store_f32=True, **kw)
        assert rel_l2(to_np(op.apply(to_dev(x))), A @ x) <= TOL64, kw
        assert rel_l2(to_np(op.apply(to_dev(x, torch.float32))), A @ x) <= TOL32, kw
        z = op.apply(torch.zeros(spec.n_dof, dtype=torch.float64, device="cuda"))
        assert float(z.abs().max()) == 0.0


# The same shapes for the Gauss kernel, whose lattice form (structured meshes)
# takes bricks of several elements along x: one element, one ragged brick, a
# column of single-element bricks.
GAUSS_EDGE_CASES = [(p, n) for p in (1, 2, 4, 6, 7) for n in ((1, 1, 1), (9, 1, 1), (1, 5, 3))]


@pytest.mark.parametrize("p,n", GAUSS_EDGE_CASES,
                         ids=[f"p{c[0]}-{c[1][0]}x{c[1][1]}x{c[1][2]}" for c in GAUSS_EDGE_CASES])
def test_apply_degenerate_meshes_gauss(p, n):
    announce(f"apply degenerate gauss p{p} {n}")
    spec = synth.slab(p, n, quad="gauss", nq1d=p + 2)
    prob, A, M, K = oracle_problem(spec)
    x = synth.uniform(107, spec.n_dof)
    for kw in (dict(), dict(structured=False)):
        op, _ = _op(spec, store_f32=True, **kw)
        assert rel_l2(to_np(op.apply(to_dev(x))), A @ x) <= TOL64, kw
        assert rel_l2(to_np(op.apply(to_dev(x, torch.float32))), A @ x) <= TOL32, kw


@pytest.mark.parametrize("quad,q", [("gll", 0), ("gauss", 4)])
@pytest.mark.parametrize("n_dof", [0, 7])
def test_empty_mesh(quad, q, n_dof):
    """No elements: A is the zero matrix on the (isolated) nodes, so every apply,
    the mass and the diagonal are zero, y += A x leaves y as it was, CG with a
    zero right-hand side stops at once, and with a nonzero one it reports the
    breakdown p^T A p = 0."""
    announce(f"empty mesh {quad} n_dof={n_dof}")
    import types
    dev = torch.device("cuda", torch.cuda.current_device())
    dofs = types.SimpleNamespace(p=2, n=(0, 0, 0), n_elem=0, n_dof=n_dof, device=dev,
                                 elem_dof=torch.empty((0, 27), dtype=torch.int32, device=dev),
                                 xyz=torch.zeros((n_dof, 3), dtype=torch.float64, device=dev),
                                 fiber=None)
    op = mf.Operator(dofs, quad=quad, nq1d=q, structured=False, store_f32=True)
    x = to_dev(synth.uniform(3, n_dof))
    for v in (x, x.float()):
        assert int(torch.count_nonzero(op.apply(v))) == 0
        assert int(torch.count_nonzero(op.apply_mass(v))) == 0
        y = torch.ones_like(v)
        op.apply_add(v, y)
        assert bool((y == 1).all())
    assert int(torch.count_nonzero(op.diagonal())) == 0
    u, info = mf.pcg(op, torch.zeros_like(x), rtol=1e-10)
    assert info.status == [0] and info.iters == [0] and int(torch.count_nonzero(u)) == 0
    if n_dof:
        u, info = mf.pcg(op, x, rtol=1e-10, check=False)
        assert info.status == [-6], info


def _row_lengths(spec, pattern):
    """Row lengths of the CSR patterns on a lattice: along each axis a node's
    elements span p + 1 nodes (2p + 1 on an interior element face); the element
    pattern holds the product of the three spans, the coupled one leaves out the
    nodes differing from the row's node in all three coordinates."""
    p = spec.p
    counts = [np.array([p + 1 if i % p else (2 * p + 1 if 0 < i < p * n else p + 1)
                        for i in range(p * n + 1)]) for n in spec.n]
    full = np.einsum("k,j,i->kji", counts[2], counts[1], counts[0]).reshape(-1)
    if pattern == "element":
        return full
    return full - np.einsum("k,j,i->kji", counts[2] - 1, counts[1] - 1, counts[0] - 1).reshape(-1)


@pytest.mark.parametrize("pattern", ["element", "coupled"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_assembled_matrix(p, pattern):
    """The matrix-based path: the CSR matrix assembled on the GPU equals the
    oracle's assembly of the element matrices, and its product the matrix-free
    apply.  The element pattern holds every node pair sharing an element; the
    coupled one only those that also share a lattice coordinate (under GLL
    collocation the others are zero, so the oracle's matrix must still be
    matched entry for entry)."""
    import scipy.sparse as sp
    announce(f"csr p{p} {pattern}")
    spec = _spec(p, (3, 2, 2) if p <= 5 else (2, 2, 1))
    prob, A, M, K = oracle_problem(spec, sigma_seed=5)
    op, _ = _op(spec, sigma=to_dev(prob.sigma))
    csr = mf.CsrMatrix(op, pattern)
    rp, col, val = csr.row_ptr.cpu().numpy(), csr.col.cpu().numpy().astype(np.int64), to_np(csr.val)
    assert rp[0] == 0 and rp[-1] == csr.nnz == len(col)
    assert np.array_equal(np.diff(rp), _row_lengths(spec, pattern))
    assert all(np.all(np.diff(col[rp[r]:rp[r + 1]]) > 0) for r in range(0, spec.n_dof, 7))
    if pattern == "coupled":
        NX, NY = p * spec.n[0] + 1, p * spec.n[1] + 1
        ijk = lambda g: (g % NX, (g // NX) % NY, g // (NX * NY))
        for r in range(0, spec.n_dof, 5):
            c = ijk(col[rp[r]:rp[r + 1]])
            share = (c[0] == ijk(r)[0]) | (c[1] == ijk(r)[1]) | (c[2] == ijk(r)[2])
            assert bool(share.all()), r
    Ag = sp.csr_matrix((val, col, rp), shape=A.shape)
    assert abs(Ag - A).max() <= 1e-13 * abs(A).max()
    x = synth.uniform(104, spec.n_dof)
    assert rel_l2(to_np(csr.apply(to_dev(x))), A @ x) <= TOL64


def test_assembled_matrix_rejects_unknown_patterns():
    """An unknown pattern code is EINVAL from the library (and a ValueError from
    the binding), with nothing written."""
    import ctypes as C
    from paper_2205_05136_amd import _lib as L
    announce("csr unknown pattern")
    op, _ = _op(_spec(2, (2, 2, 1)))
    nnz = C.c_int64(-5)
    assert L.load().mfsem_csr_nnz(op.handle, 2, C.byref(nnz)) == -1 and nnz.value == -5
    assert L.load().mfsem_csr_nnz(op.handle, -1, C.byref(nnz)) == -1 and nnz.value == -5
    with pytest.raises(ValueError):
        mf.CsrMatrix(op, "full")


def test_assembled_matrix_patterns_agree_at_full_size():
    """On the 229,425-DOF c2 slab at p = 4 (the matrix-based comparison's mesh):
    both patterns have their closed-form sizes, the coupled one holds every
    non-zero of the element pattern, and the two products agree."""
    announce("csr patterns c2")
    spec = synth.C2
    op, _ = _op(spec)
    full, cpl = mf.CsrMatrix(op, "element"), mf.CsrMatrix(op, "coupled")
    assert full.nnz == int(_row_lengths(spec, "element").sum())
    assert cpl.nnz == int(_row_lengths(spec, "coupled").sum())
    assert int(torch.count_nonzero(full.val)) == int(torch.count_nonzero(cpl.val))
    x = to_dev(synth.uniform(105, spec.n_dof))
    y1, y2 = full.apply(x), cpl.apply(x)
    assert float(torch.linalg.norm(y1 - y2)) <= 1e-14 * float(torch.linalg.norm(y1))
    assert rel_l2(to_np(y1), to_np(op.apply(x))) <= TOL64


@pytest.mark.parametrize("p,quad,q", [(2, "gll", 0), (4, "gll", 0), (5, "gll", 0), (6, "gll", 0),
                                      (7, "gll", 0), (2, "gauss", 4), (4, "gauss", 6),
                                      (7, "gauss", 9)])
def test_apply_f32(p, quad, q):
    announce(f"apply f32 p{p} {quad}")
    spec = _spec(p, quad=quad, nq1d=q)
    prob, A, M, K = oracle_problem(spec)
    op, _ = _op(spec, store_f32=True)
    x = synth.uniform(101, spec.n_dof)
    y = to_np(op.apply(to_dev(x, torch.float32)))
    assert rel_l2(y, A @ x) <= TOL32
    d = to_np(op.diagonal(torch.float32))
    assert rel_l2(d, A.diagonal()) <= TOL32


@pytest.mark.parametrize("p,quad,q,n", [(3, "gll", 0, (5, 3, 2)), (3, "gauss", 5, (5, 3, 2)),
                                        (4, "gauss", 6, (4, 3, 2)), (7, "gauss", 9, (2, 2, 1))])
def test_apply_singular_sigma(p, quad, q, n):
    """sigma_t = 0 makes sigma = sigma_l f f^T singular: det G = 0, so the mass
    weight cannot be recovered from it and the kernels read the stored W|J|
    (for Gauss from p = 4 in FP64 through the flux loop's stored-weight copy)."""
    announce(f"apply singular sigma p{p} {quad}")
    spec = _spec(p, n, quad=quad, nq1d=q).with_(sigma=(0.17, 0.0, 0.0))
    prob, A, M, K = oracle_problem(spec)
    x = synth.uniform(106, spec.n_dof)
    kws = (dict(), dict(structured=False)) if quad == "gll" else (dict(),)
    for kw in kws:
        op, _ = _op(spec, store_f32=True, **kw)
        assert rel_l2(to_np(op.apply(to_dev(x))), A @ x) <= TOL64, kw
        assert rel_l2(to_np(op.apply(to_dev(x, torch.float32))), A @ x) <= TOL32, kw
        assert rel_l2(to_np(op.apply_mass(to_dev(x))), M @ x) <= TOL64, kw


def test_apply_batch_sigma():
    announce("apply batch of 3 sigma sets")
    spec = _spec(3, (4, 3, 2))
    sig = synth.element_sigma(31, 3, spec.n_elem)
    box = mf.Box.from_spec(spec)
    op = mf.Operator.from_spec(spec, box=box, sigma=to_dev(sig))
    x = synth.uniform(102, (3, spec.n_dof))
    y = to_np(op.apply(to_dev(x)))
    otf = mf.Operator.from_spec(spec, box=box, sigma=to_dev(sig), geom="onthefly")
    y_otf = to_np(otf.apply(to_dev(x)))
    for b in range(3):
        A, _, _ = oop.Problem(spec, sigma=sig[b]).assemble()
        assert rel_l2(y[b], A @ x[b]) <= TOL64
        assert rel_l2(y_otf[b], A @ x[b]) <= TOL64
    # set_sigma recomputes the geometry
    sig2 = sig[::-1].copy()
    op.set_sigma(to_dev(sig2))
    y2 = to_np(op.apply(to_dev(x)))
    A0, _, _ = oop.Problem(spec, sigma=sig2[0]).assemble()
    assert rel_l2(y2[0], A0 @ x[0]) <= TOL64


@pytest.mark.parametrize("p,q", [(3, 5), (5, 7)])
def test_apply_batch_sigma_gauss(p, q):
    """The SEM (Gauss) kernels over a batch of 3 per-element sigma sets, FP64 and
    FP32, the diagonal and the mass of every member against the oracle."""
    announce(f"apply gauss batch of 3 sigma sets p={p} q={q}")
    spec = _spec(p, (4, 3, 2), quad="gauss", nq1d=q)
    sig = synth.element_sigma(37 + p, 3, spec.n_elem)
    op = mf.Operator.from_spec(spec, sigma=to_dev(sig), store_f32=True)
    x = synth.uniform(104 + p, (3, spec.n_dof))
    y = to_np(op.apply(to_dev(x)))
    y32 = to_np(op.apply(to_dev(x, torch.float32)))
    d = to_np(op.diagonal())
    m = to_np(op.apply_mass(to_dev(x)))
    for b in range(3):
        A, M, _ = oop.Problem(spec, sigma=sig[b]).assemble()
        assert rel_l2(y[b], A @ x[b]) <= TOL64, b
        assert rel_l2(y32[b], A @ x[b]) <= TOL32, b
        assert rel_l2(d[b], A.diagonal()) <= TOL64, b
        assert rel_l2(m[b], M @ x[b]) <= TOL64, b


@pytest.mark.parametrize("p,n", [(5, (9, 2, 2)), (6, (8, 1, 2)), (7, (3, 1, 3))])
def test_apply_batch_ragged_bricks_f64_f32(p, n):
    """Batched applies (two sigma sets) on meshes whose last lattice brick is
    partial along x and z, in FP64 and FP32, so that the lanes outside the mesh
    (which load from a clamped address and discard the value) are exercised in
    both load orders of the lattice kernel."""
    announce(f"apply batch 2 ragged bricks p={p} n={n}")
    spec = _spec(p, n)
    sig = synth.element_sigma(41 + p, 2, spec.n_elem)
    op = mf.Operator.from_spec(spec, sigma=to_dev(sig), store_f32=True)
    x = synth.uniform(103 + p, (2, spec.n_dof))
    y64 = to_np(op.apply(to_dev(x)))
    y32 = to_np(op.apply(to_dev(x, torch.float32)))
    for b in range(2):
        A, _, _ = oop.Problem(spec, sigma=sig[b]).assemble()
        ref = A @ x[b]
        assert rel_l2(y64[b], ref) <= TOL64, b
        assert rel_l2(y32[b], ref) <= TOL32, b


def test_apply_sheet_orthotropic():
    """Full orthotropic tensor with a sheet field (sigma_n != sigma_t)."""
    announce("apply orthotropic sheet")
    spec = _spec(3, (3, 2, 2)).with_(sigma=(0.17, 0.05, 0.019))
    box = mf.Box.from_spec(spec)
    m = omesh.box(spec)
    sheet = np.stack([-m.fiber[:, 1], m.fiber[:, 0], 0.3 * np.ones(spec.n_dof)], axis=1)
    op = mf.Operator.from_spec(spec, box=box, sheet=to_dev(sheet))
    # oracle with the sheet: assemble through element_matrices
    prob = oop.Problem(spec)
    x = synth.uniform(103, spec.n_dof)
    y_ref = np.zeros(spec.n_dof)
    for el in prob.chunks():
        X = prob.mesh.xyz[prob.mesh.elem_dof[el]]
        geo = oop.geometry(X, prob.mesh.fiber[prob.mesh.elem_dof[el]],
                           sheet[prob.mesh.elem_dof[el]], spec.p, prob.pts, prob.w)
        Me, Ke = oop.element_matrices(geo, prob.sigma[el], spec.p, prob.pts, spec.alpha)
        ye = np.einsum("eij,ej->ei", spec.alpha * Me + Ke, x[prob.elem_dof[el]])
        np.add.at(y_ref, prob.elem_dof[el].reshape(-1), ye.reshape(-1))
    assert rel_l2(to_np(op.apply(to_dev(x))), y_ref) <= TOL64


@pytest.mark.parametrize("quad", ["gll", "gauss"])
def test_paper_slab_shape_sheet_hierarchy(quad):
    """The paper-shaped workload's set-up at a small size: orthotropic tensor from
    the spec's sheet, p- then h-coarsening, Chebyshev degree 5; apply, V-cycle and
    PCG against the oracle."""
    announce(f"paper-slab shape {quad}")
    spec = synth.paper_slab(2, quad=quad).with_(n=(8, 4, 4))
    chain = (("p", 1), ("h",))
    probs, mats, Ps = _levels_oracle(spec, chain)
    ops, mg = mf.hierarchy(spec, coarsening=chain, degree=5)
    for l, op in enumerate(ops):
        x = synth.uniform(410 + l, op.n_dof)
        assert rel_l2(to_np(op.apply(to_dev(x))), mats[l] @ x) <= TOL64
    lam = mg.lambdas().numpy()[:, 0]
    levels = [(A, 1 / A.diagonal(), float(l)) for A, l in zip(mats, lam)]
    b = synth.uniform(510, spec.n_dof)
    assert rel_l2(to_np(mg.vcycle(to_dev(b))), osol.vcycle(levels, Ps, b, 5, 10)) <= TOL64
    u, info = mf.pcg(ops[0], to_dev(b), mg=mg, rtol=1e-12, max_it=100)
    assert np.linalg.norm(b - mats[0] @ to_np(u)) <= 1.01e-12 * np.linalg.norm(b)


# -------------------------------------------------------------- multigrid ---
def _levels_oracle(spec, chain):
    """Oracle level matrices and prolongations for a coarsening chain (levels
    below the finest use GLL quadrature, SEM-NI, as the library's hierarchy)."""
    probs = [oop.Problem(spec)]
    Ps = []
    cur, n, p = spec, spec.n, spec.p
    for step in chain:
        if step[0] == "p":
            probs.append(oop.Problem(cur, dof_p=step[1], quad="gll"))
            Ps.append(omg.prolongation_p(n, p, step[1]))
            p = step[1]
        else:
            nc = tuple(k // 2 for k in n)
            Ps.append(omg.prolongation_h(n, p))
            cur = cur.with_(n=nc, shear_amp=cur.shear_amp / 2, p=p, quad="gll", nq1d=0)
            probs.append(oop.Problem(cur))
            n = nc
    mats = [pr.assemble()[0] for pr in probs]
    return probs, mats, Ps


CHAINS = {
    "p4-2-1": (_spec(4, (4, 3, 2)), (("p", 2), ("p", 1))),
    "h-p3": (_spec(3, (4, 2, 4)), (("h",), ("p", 1))),
    "p7-3-1": (_spec(7, (2, 2, 1)), (("p", 3), ("p", 1))),
}


@pytest.mark.parametrize("structured", [True, False], ids=["lattice", "elements"])
@pytest.mark.parametrize("name", list(CHAINS))
def test_transfers(name, structured):
    """Prolongation and restriction against the oracle's matrices, both as 1D
    lattice passes (structured levels) and per element (general meshes)."""
    announce(f"transfers {name} structured={structured}")
    spec, chain = CHAINS[name]
    probs, mats, Ps = _levels_oracle(spec, chain)
    ops, mg = mf.hierarchy(spec, coarsening=chain, lambda_max=[1.0] * len(mats),
                           structured=structured)
    for l, P in enumerate(Ps):
        xc = synth.uniform(200 + l, P.shape[1])
        rf = synth.uniform(300 + l, P.shape[0])
        assert rel_l2(to_np(mg.prolong(l, to_dev(xc))), P @ xc) <= TOL64
        assert rel_l2(to_np(mg.restrict(l, to_dev(rf))), P.T @ rf) <= TOL64
    for l, op in enumerate(ops):
        x = synth.uniform(400 + l, op.n_dof)
        assert rel_l2(to_np(op.apply(to_dev(x))), mats[l] @ x) <= TOL64


@pytest.mark.parametrize("structured", [True, False], ids=["lattice", "elements"])
def test_transfers_f32_batched(structured):
    """FP32 transfers of a batch of two (per-member sigma) against the oracle."""
    announce(f"transfers f32 batch 2 structured={structured}")
    spec, chain = CHAINS["p4-2-1"]
    probs, mats, Ps = _levels_oracle(spec, chain)
    sig = synth.element_sigma(210, 2, spec.n_elem)
    ops, mg = mf.hierarchy(spec, coarsening=chain, lambda_max=[1.0] * 2 * len(mats),
                           sigma=to_dev(sig), precision=torch.float32, structured=structured)
    for l, P in enumerate(Ps):
        xc = synth.uniform(220 + l, (2, P.shape[1]))
        rf = synth.uniform(230 + l, (2, P.shape[0]))
        yp = to_np(mg.prolong(l, to_dev(xc, torch.float32)))
        yr = to_np(mg.restrict(l, to_dev(rf, torch.float32)))
        for b in range(2):
            assert rel_l2(yp[b], P @ xc[b]) <= TOL32
            assert rel_l2(yr[b], P.T @ rf[b]) <= TOL32


@pytest.mark.parametrize("structured", [True, False], ids=["lattice", "elements"])
@pytest.mark.parametrize("name", list(CHAINS))
def test_vcycle_matches_oracle(name, structured):
    announce(f"vcycle {name} structured={structured}")
    spec, chain = CHAINS[name]
    probs, mats, Ps = _levels_oracle(spec, chain)
    lam = [1.05 * osol.lanczos_lambda_max(A, 1 / A.diagonal(), synth.uniform(7, A.shape[0]))
           for A in mats]
    levels = [(A, 1 / A.diagonal(), l) for A, l in zip(mats, lam)]
    ops, mg = mf.hierarchy(spec, coarsening=chain, lambda_max=lam, degree=3, coarse_degree=6,
                           structured=structured)
    b = synth.uniform(500, spec.n_dof)
    z_ref = osol.vcycle(levels, Ps, b, 3, 6)
    z = to_np(mg.vcycle(to_dev(b)))
    assert rel_l2(z, z_ref) <= TOL64
    # cycles in a row: the work buffers must come back to their zero state
    b2 = synth.uniform(501, spec.n_dof)
    assert rel_l2(to_np(mg.vcycle(to_dev(b2))), osol.vcycle(levels, Ps, b2, 3, 6)) <= TOL64
    assert rel_l2(to_np(mg.vcycle(to_dev(b))), z_ref) <= TOL64


@pytest.mark.parametrize("prec", [torch.float64, torch.float32])
def test_vcycle_graph_replays_match_launches(prec):
    """V-cycles replayed from captured HIP graphs equal plain launches: several
    replays with other work and synchronisations between them, two (r, z) pairs,
    and a change of alpha on the levels (which must be captured anew)."""
    announce(f"vcycle graphs {prec}")
    spec, chain = CHAINS["p4-2-1"]
    ops, mg_g = mf.hierarchy(spec, coarsening=chain, degree=3, precision=prec)
    mg_e = mf.Multigrid(ops, mg_g.transfers, degree=3, precision=prec, graphs=False,
                        lambda_max=mg_g.lambdas().reshape(-1))
    mg_g = mf.Multigrid(ops, mg_g.transfers, degree=3, precision=prec, graphs=True,
                        lambda_max=mg_g.lambdas().reshape(-1))
    tol = 1e-13 if prec == torch.float64 else 1e-6
    rs = [to_dev(synth.uniform(600 + i, spec.n_dof), prec) for i in range(3)]
    zs = [torch.empty_like(rs[0]) for _ in range(2)]
    for rep in range(4):
        for k, r in enumerate(rs):
            z = zs[k % 2]
            mg_g.vcycle(r, out=z)
            ze = mg_e.vcycle(r)
            torch.cuda.synchronize()
            assert rel_l2(to_np(z), to_np(ze)) <= tol, (rep, k)
            ops[0].apply(to_dev(synth.uniform(700 + rep, spec.n_dof)))  # other work between
        if rep == 2:
            for op in ops:
                op.set_alpha(0.5 * op.alpha)


def test_lambda_estimate_bounds():
    announce("lambda estimate")
    spec, chain = CHAINS["p4-2-1"]
    probs, mats, Ps = _levels_oracle(spec, chain)
    ops, mg = mf.hierarchy(spec, coarsening=chain)
    lam = mg.lambdas().numpy()[:, 0]
    for A, l in zip(mats, lam):
        d = A.diagonal()
        S = (A.multiply(1 / np.sqrt(d)[:, None]).multiply(1 / np.sqrt(d)[None, :])).toarray()
        emax = np.linalg.eigvalsh(S).max()
        assert l <= emax * (1 + 1e-10) and l >= 0.8 * emax, (l, emax)


# ------------------------------------------------------------------ solves ---
def test_cg_c1():
    announce("cg c1")
    spec = synth.C1
    prob, A, M, K = oracle_problem(spec)
    op, _ = _op(spec)
    f = synth.uniform(1, spec.n_dof)
    x, info = mf.pcg(op, to_dev(f), rtol=1e-14, max_it=500)
    x_ref = spla.spsolve(A.tocsc(), f)
    assert rel_l2(to_np(x), x_ref) <= TOL64
    assert info.status == [0]
    # the benchmark's relative tolerance 1e-10 from x0 = 0
    x10, info10 = mf.pcg(op, to_dev(f), rtol=1e-10, max_it=500)
    r = f - A @ to_np(x10)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(f)


@pytest.mark.parametrize("name", ["p4-2-1", "h-p3"])
def test_gmg_pcg(name):
    announce(f"gmg pcg {name}")
    spec, chain = CHAINS[name]
    A = oracle_problem(spec)[1]
    f = synth.uniform(2, spec.n_dof)
    x_ref = spla.spsolve(A.tocsc(), f)
    ops, mg = mf.hierarchy(spec, coarsening=chain, degree=3)
    x, info = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-14, max_it=200)
    assert rel_l2(to_np(x), x_ref) <= TOL64
    assert info.iters[0] <= 30
    x0, info0 = mf.pcg(ops[0], to_dev(f), rtol=1e-14, max_it=5000)
    assert info.iters[0] < info0.iters[0]


def test_mixed_precision_pcg():
    announce("mixed pcg")
    spec, chain = CHAINS["p4-2-1"]
    A = oracle_problem(spec)[1]
    f = synth.uniform(3, spec.n_dof)
    x_ref = spla.spsolve(A.tocsc(), f)
    ops, mg = mf.hierarchy(spec, coarsening=chain, degree=3, precision=torch.float32)
    x, info = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-10, max_it=200)
    assert info.status == [0]
    assert rel_l2(to_np(x), x_ref) <= 1e-8
    x2, info2 = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-14, max_it=200)
    assert rel_l2(to_np(x2), x_ref) <= TOL64


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("flexible", [False, True])
def test_pcg_variants(precision, flexible):
    """Standard and flexible CG around the FP64 and the FP32 V-cycle (and the
    unpreconditioned loop in both forms): every combination reaches the direct
    solution, and the preconditioned ones in a few dozen iterations."""
    announce(f"pcg {precision} flexible={flexible}")
    spec, chain = CHAINS["p4-2-1"]
    A = oracle_problem(spec)[1]
    f = synth.uniform(7, spec.n_dof)
    x_ref = spla.spsolve(A.tocsc(), f)
    dt = torch.float64 if precision == "f64" else torch.float32
    ops, mg = mf.hierarchy(spec, coarsening=chain, degree=3, precision=dt)
    # standard CG assumes a symmetric preconditioner, which the FP32 V-cycle is
    # only to single precision: it is held to the mixed-precision bar
    rtol, bar = (1e-10, 1e-8) if (precision == "f32" and not flexible) else (1e-13, 1e-11)
    x, info = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=rtol, max_it=300, flexible=flexible)
    assert info.status == [0], info.status
    assert info.iters[0] <= 60, info.iters
    assert rel_l2(to_np(x), x_ref) <= bar
    if precision == "f64":
        x0, info0 = mf.pcg(ops[0], to_dev(f), rtol=1e-13, max_it=5000, flexible=flexible)
        assert info0.status == [0]
        assert rel_l2(to_np(x0), x_ref) <= 1e-11


# The c3 hierarchy (Section 3: SEM with Gauss points, here q = p + 2 = 9, or
# SEM-NI; Section 4.3: p-multigrid) at reduced size: a 4 x 3 x 2 element piece
# of the c3 slab at its element edges (20/128, 7/48, 3/24 mm), p = 7 (9,570
# DOFs), with the chain 7 -> 5 -> 3 -> 1 the benchmark uses at 51M DOFs.
_C3_N = (4, 3, 2)
_C3_LEN = tuple(k * L / m for k, L, m in zip(_C3_N, synth.SLAB_LEN, synth.C3_NI.n))
C3_SMALL = {"gll-q8": synth.C3_NI.with_(n=_C3_N, length=_C3_LEN),
            "gauss-q9": synth.C3_SEM.with_(n=_C3_N, length=_C3_LEN)}
C3_CHAIN = (("p", 5), ("p", 3), ("p", 1))


@pytest.mark.parametrize("name", list(C3_SMALL))
def test_c3_reduced_solves(name):
    """FP64 GMG-PCG and the mixed-precision FCG (FP32 V-cycle) on the c3
    hierarchy against the oracle's direct solve: 1e-12 when solved to 1e-14;
    at the benchmark's 1e-10 the true residual of the oracle's matrix is within
    the tolerance and the mixed solution within 1e-8 of the oracle's."""
    announce(f"c3 reduced solves {name}")
    spec = C3_SMALL[name]
    A = oracle_problem(spec)[1]
    f = synth.uniform(3, spec.n_dof)
    x_ref = spla.spsolve(A.tocsc(), f)
    nf = np.linalg.norm(f)
    for precision in (torch.float64, torch.float32):
        ops, mg = mf.hierarchy(spec, coarsening=C3_CHAIN, degree=3, precision=precision)
        x, info = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-14, max_it=200)
        assert info.status == [0] and info.iters[0] <= 40, info.iters
        assert rel_l2(to_np(x), x_ref) <= TOL64, precision
        x10, info10 = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-10, max_it=200)
        assert info10.status == [0]
        assert np.linalg.norm(f - A @ to_np(x10)) <= 1.01e-10 * nf
        assert rel_l2(to_np(x10), x_ref) <= 1e-8


def test_batched_pcg_and_grad():
    announce("batched pcg + grad")
    spec = synth.BoxSpec(p=3, n=(3, 3, 2), length=(1.5, 1.5, 1.0), fiber=True,
                         theta0=-1.0, theta1=1.0, sigma=synth.SLAB_SIGMA, alpha=28.0)
    sig = synth.element_sigma(4, 2, spec.n_elem)
    box = mf.Box.from_spec(spec)
    op = mf.Operator.from_spec(spec, box=box, sigma=to_dev(sig))
    f = synth.uniform(5, (2, spec.n_dof))
    x, info = mf.pcg(op, to_dev(f), rtol=1e-14, max_it=2000)
    for b in range(2):
        prob = oop.Problem(spec, sigma=sig[b])
        A, _, _ = prob.assemble()
        assert rel_l2(to_np(x)[b], spla.spsolve(A.tocsc(), f[b])) <= TOL64
        u = synth.uniform(6 + b, spec.n_dof)
        w = synth.uniform(8 + b, spec.n_dof)
        g_ref = oadj.grad_sigma(prob, u, w)
        uu = np.stack([u if bb == b else np.zeros_like(u) for bb in range(2)])
        ww = np.stack([w if bb == b else np.zeros_like(w) for bb in range(2)])
        g = to_np(op.grad_sigma(to_dev(uu), to_dev(ww)))[b]
        assert rel_l2(g, g_ref) <= TOL64


def test_c4_shaped_batch8_solve_and_grad():
    """The c4 workload's shape at reduced size: a p = 4 box at the c4 element
    edge (0.5 mm) with the c4 fiber, 8 per-element conductivity sets drawn as
    in c4, one batched GMG-PCG solve of all 8 and the dL/dsigma contraction of
    all 8 in one launch, each member against the oracle (1e-12)."""
    announce("c4-shaped batch 8")
    spec = synth.C4.with_(n=(3, 3, 2), length=(1.5, 1.5, 1.0))
    B = 8
    sig = synth.element_sigma(4, B, spec.n_elem)
    ops, mg = mf.hierarchy(spec, coarsening=(("p", 2), ("p", 1)), degree=3, sigma=to_dev(sig))
    f = synth.uniform(5, (B, spec.n_dof))
    x, info = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-14, max_it=300)
    assert info.status == [0] * B
    u = synth.uniform(6, (B, spec.n_dof))
    w = synth.uniform(7, (B, spec.n_dof))
    g = to_np(ops[0].grad_sigma(to_dev(u), to_dev(w)))
    xs = to_np(x)
    for b in range(B):
        prob = oop.Problem(spec, sigma=sig[b])
        A, _, _ = prob.assemble()
        assert rel_l2(xs[b], spla.spsolve(A.tocsc(), f[b])) <= TOL64, b
        assert rel_l2(g[b], oadj.grad_sigma(prob, u[b], w[b])) <= TOL64, b


GRAD_CASES = {
    "fiber-p3": synth.BoxSpec(p=3, n=(3, 2, 2), length=(1.5, 1.0, 1.0), fiber=True, theta0=-1.0,
                              theta1=1.0, sigma=(0.17, 0.03, 0.03), alpha=2.0),
    "sheet-p2": synth.paper_slab(2).with_(n=(3, 2, 2), theta0=-0.4, theta1=0.9),
    "isotropic-p4": synth.BoxSpec(p=4, n=(2, 2, 1), sigma=(0.2, 0.2, 0.2), alpha=1.0),
    "gauss-p3-q5": synth.slab(3, (3, 2, 2), quad="gauss", nq1d=5),
    "sheared-p5": synth.slab(5, (2, 2, 1)),
    "direct-sum-p7": synth.slab(7, (2, 1, 1)),
}


@pytest.mark.parametrize("name", list(GRAD_CASES))
def test_grad_sigma_cases(name):
    """dA/dsigma contracted with two vectors, per element, against the oracle:
    fiber only, fiber and sheet, no fiber, Gauss points, a sheared map, and a
    degree whose arrays exceed the sum-factorised kernel's LDS budget."""
    announce(f"grad sigma {name}")
    spec = GRAD_CASES[name]
    sig = synth.element_sigma(30, 2, spec.n_elem)
    sig[..., 2] = sig[..., 1] * 0.6  # distinct sigma_n (used with a sheet)
    op = mf.Operator.from_spec(spec, sigma=to_dev(sig))
    u = synth.uniform(31, (2, spec.n_dof))
    w = synth.uniform(32, (2, spec.n_dof))
    g = to_np(op.grad_sigma(to_dev(u), to_dev(w)))
    for b in range(2):
        prob = oop.Problem(spec, sigma=sig[b])
        g_ref = oadj.grad_sigma(prob, u[b], w[b])
        assert rel_l2(g[b], g_ref) <= TOL64, b
    # the scale argument multiplies the result (the solve's adjoint takes -1)
    gs = to_np(op.grad_sigma(to_dev(u), to_dev(w), scale=-2.5))
    assert np.array_equal(gs, -2.5 * g)


def test_ionic_step():
    announce("ionic step")
    n = 5000
    V = synth.uniform(9, n, -85.0, 30.0)
    w = synth.uniform(10, n, 0.0, 1.5)
    ist = synth.uniform(11, n, 0.0, 50.0)
    m = synth.uniform(12, n, 0.1, 1.0)
    b_ref, w_ref = oion.imex_rhs_and_gate(V, w, ist, m, 0.05, synth.CHI, synth.CM, synth.AP_PARAMS)
    wd = to_dev(w)
    b = mf.ap_imex_rhs(to_dev(V), wd, to_dev(m), 0.05, synth.CHI, synth.CM, synth.AP_PARAMS,
                       i_stim=to_dev(ist))
    assert rel_l2(to_np(b), b_ref) <= 1e-14
    assert rel_l2(to_np(wd), w_ref) <= 1e-14


def test_ionic_bdf2_step():
    announce("ionic bdf2 step")
    n = 5000
    V = synth.uniform(13, n, -85.0, 30.0)
    Vo = V + synth.uniform(14, n, -3.0, 3.0)
    w = synth.uniform(15, n, 0.0, 1.5)
    wo = w + synth.uniform(16, n, -0.05, 0.05)
    ist = synth.uniform(17, n, 0.0, 50.0)
    m = synth.uniform(18, n, 0.1, 1.0)
    dt = 0.05
    b_ref, w_ref = oion.bdf2_rhs_and_gate(V, Vo, w, wo, ist, m, dt, synth.CHI, synth.CM,
                                          synth.AP_PARAMS)
    wd, wod = to_dev(w), to_dev(wo)
    b = mf.ap_bdf2_rhs(to_dev(V), to_dev(Vo), wd, wod, to_dev(m), dt, synth.CHI, synth.CM,
                       synth.AP_PARAMS, i_stim=to_dev(ist))
    assert rel_l2(to_np(b), b_ref) <= 1e-14
    assert rel_l2(to_np(wd), w_ref) <= 1e-14
    assert np.array_equal(to_np(wod), w)  # w_old <- w^n


def test_activation_update():
    """Activation times (Section 5.1: the time of the largest |dV/dt|) kept as a
    running maximum, and the separately named level crossing, bit-exact against
    the oracle over a series of steps: the decision |V - V_old|/dt > rate is an
    FP64 division and comparison on both sides.  The potentials are small
    integers, so many steps tie exactly and the earliest must be kept; half the
    nodes sit near -40 mV so that crossings occur; the series is generated
    stepwise from seeded draws."""
    announce("activation update")
    n, steps, dt = 4099, 12, 0.125
    act, rate, cross = np.full(n, -1.0), np.zeros(n), np.full(n, -1.0)
    actd, rated, crossd = to_dev(act), to_dev(rate), to_dev(cross)
    V = np.round(synth.uniform(13, n, -80.0, -20.0))
    t = 0.0
    for k in range(steps):
        Vn = V + np.round(synth.uniform(200 + k, n, -6.0, 6.0))
        Vn[::7] = V[::7]  # nodes that do not move in this step
        t += dt
        act, rate = oion.activation_update(act, rate, V, Vn, t, dt)
        cross = oion.threshold_crossing_update(cross, V, Vn, t - dt, t, -40.0)
        mf.activation_update(to_dev(Vn), to_dev(V), t, dt, act=actd, rate=rated, v_cross=-40.0,
                             cross=crossd)
        V = Vn
    assert np.array_equal(to_np(actd), act) and np.array_equal(to_np(rated), rate)
    assert np.array_equal(to_np(crossd), cross)
    assert (cross > 0).sum() > 100 and (act > 0).sum() > n // 2
    # without the crossing output, and an argument error
    act2 = to_dev(np.full(n, -1.0))
    rate2 = to_dev(np.zeros(n))
    mf.activation_update(to_dev(V), to_dev(V - 1.0), 1.0, dt, act=act2, rate=rate2)
    assert float(act2.min()) == float(act2.max()) == 1.0 - 0.5 * dt
    with pytest.raises(mf.MfsemError):
        mf.activation_update(to_dev(V), to_dev(V), 1.0, dt, act=act2, rate=None)


# ------------------------------------------------------------------ errors ---
def test_error_paths():
    announce("error paths")
    spec = _spec(2, (2, 2, 2))
    box = mf.Box.from_spec(spec)
    bad = box.xyz.clone()
    bad[:, 0] = -bad[:, 0]  # mirrored map: det J < 0 everywhere
    with pytest.raises(mf.MfsemError) as e:
        mf.Operator.from_spec(spec, box=box, xyz=bad)
    assert e.value.status == -3 and "element 0" in str(e.value)
    with pytest.raises(mf.MfsemError) as e:
        mf.Operator.from_spec(spec, box=box, quad="gll", nq1d=spec.p + 2)
    assert e.value.status == -1
    # on-the-fly geometry refused where it does not apply (Gauss points, p = 7)
    with pytest.raises(mf.MfsemError) as e:
        mf.Operator.from_spec(spec, box=box, quad="gauss", nq1d=spec.p + 1, geom="onthefly")
    assert e.value.status == -1 and "on-the-fly" in str(e.value)
    spec7 = _spec(7, (1, 1, 1))
    with pytest.raises(mf.MfsemError) as e:
        mf.Operator.from_spec(spec7, geom="onthefly")
    assert e.value.status == -1
    op = mf.Operator.from_spec(spec, box=box)
    f = to_dev(synth.uniform(1, spec.n_dof))
    x, info = mf.pcg(op, f, rtol=1e-14, max_it=1, check=False)
    assert info.status == [-5] and info.iters == [1]
    with pytest.raises(mf.MfsemError):
        mf.pcg(op, f, rtol=1e-14, max_it=1)
    fn = f.clone()
    fn[3] = float("nan")
    x, info = mf.pcg(op, fn, rtol=1e-10, max_it=10, check=False)
    assert info.status == [-7]
    with pytest.raises(ValueError):
        op.apply(torch.zeros(3, device="cuda", dtype=torch.float64))
    with pytest.raises(mf.MfsemError):
        op.apply(torch.zeros(spec.n_dof, device="cuda", dtype=torch.float32))  # no FP32 geometry
    # h-transfer arrays are range-checked on the device before any transfer uses them
    coarse = mf.Operator.from_spec(spec.with_(n=(1, 1, 1)))
    par, chi = mf.box_parents(spec.n)
    for bad_par, bad_chi in ((par + 1, chi), (par, chi + 8)):
        with pytest.raises(mf.MfsemError) as e:
            mf.Multigrid([op, coarse], [("h", bad_par.contiguous(), bad_chi.contiguous())],
                         lambda_max=[1.0, 1.0])
        assert e.value.status == -1 and "out of range" in str(e.value)
    with pytest.raises(ValueError):
        mf.Multigrid([op, coarse], [("h", par.long(), chi)], lambda_max=[1.0, 1.0])
