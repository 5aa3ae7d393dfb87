"""Meshes given by arrays (paper_2205_05136_amd.meshops): element orientation,
renumbering and locality order.  CPU: the operator the oracle assembles from
the element matrices of a rotated, shuffled and renumbered copy of a slab is
the permuted operator of the slab.  GPU: the general element kernel and a
p-multigrid PCG on such a mesh match the permuted oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import operator as oop
from paper_2205_05136_amd import meshops

SPEC = synth.slab(3, (4, 3, 2))


def _scrambled(spec, seed):
    """The slab's oracle mesh with random element rotations, element order and
    node numbering; returns (elem_dof, xyz, fiber, node_perm, elem_perm, rot)."""
    prob = oop.Problem(spec)
    m = prob.mesh
    rng = np.random.default_rng(seed)
    rot = rng.integers(0, 24, spec.n_elem)
    node_perm = rng.permutation(spec.n_dof)
    elem_perm = rng.permutation(spec.n_elem)
    ed = meshops.reorient(m.elem_dof, spec.p, rot)
    ed, xyz, fib = meshops.permute(ed, m.xyz, m.fiber, node_perm, elem_perm)
    return prob, ed, xyz, fib, node_perm, elem_perm, rot


def _assemble(prob, spec, ed, xyz, fib, sigma):
    """Oracle assembly from per-element geometry on an arbitrary element map."""
    geo = oop.geometry(xyz[ed], fib[ed], None, spec.p, prob.pts, prob.w)
    Me, Ke = oop.element_matrices(geo, sigma, spec.p, prob.pts, spec.alpha)
    Ae = spec.alpha * Me + Ke
    rows = np.repeat(ed, ed.shape[1], axis=1).reshape(-1)
    cols = np.tile(ed, (1, ed.shape[1])).reshape(-1)
    return sp.coo_matrix((Ae.reshape(-1), (rows, cols)), shape=(spec.n_dof,) * 2).tocsr()


def test_rotations_are_the_24_proper_ones():
    R = meshops.cube_rotations()
    assert len(R) == 24
    keys = {r.tobytes() for r in R}
    assert len(keys) == 24
    for a in R:
        assert round(np.linalg.det(a)) == 1
        for b in R:
            assert (a @ b).tobytes() in keys  # a group
    maps = meshops.local_rotation_maps(3)
    for mp in maps:
        assert np.array_equal(np.sort(mp), np.arange(64))  # permutations of the local nodes
    ident = [i for i, r in enumerate(R) if np.array_equal(r, np.eye(3, dtype=np.int64))]
    assert np.array_equal(maps[ident[0]], np.arange(64))


def test_scrambled_mesh_gives_the_permuted_operator():
    prob, ed, xyz, fib, node_perm, elem_perm, rot = _scrambled(SPEC, 7)
    assert len(set(rot.tolist())) > 10
    A = prob.assemble()[0]
    Au = _assemble(prob, SPEC, ed, xyz, fib, prob.sigma[elem_perm])
    Pm = sp.csr_matrix((np.ones(SPEC.n_dof), (node_perm, np.arange(SPEC.n_dof))),
                       shape=(SPEC.n_dof,) * 2)
    assert abs(Au - Pm @ A @ Pm.T).max() <= 1e-13 * abs(A).max()


def test_locality_order_is_a_renumbering():
    from oracle import mesh as omesh
    spec = synth.slab(2, (24, 12, 8))
    m = omesh.box(spec)
    rng = np.random.default_rng(8)
    ed, xyz, fib = meshops.permute(meshops.reorient(m.elem_dof, 2, rng.integers(0, 24, spec.n_elem)),
                                   m.xyz, m.fiber, rng.permutation(spec.n_dof),
                                   rng.permutation(spec.n_elem))
    node_perm, elem_perm = meshops.locality_order(ed, xyz)
    assert np.array_equal(np.sort(node_perm), np.arange(spec.n_dof))
    assert np.array_equal(np.sort(elem_perm), np.arange(spec.n_elem))
    ed2, xyz2, fib2 = meshops.permute(ed, xyz, fib, node_perm, elem_perm)
    # nodes are numbered by first appearance along the element order
    first = ed2.reshape(-1)
    _, idx = np.unique(first, return_index=True)
    assert np.all(np.diff(first[np.sort(idx)]) == 1)
    # the ordered mesh's elements sit closer to their neighbours in index than the scrambled
    cen = lambda e, x: x[e].mean(axis=1)
    d_before = np.linalg.norm(np.diff(cen(ed, xyz), axis=0), axis=1).mean()
    d_after = np.linalg.norm(np.diff(cen(ed2, xyz2), axis=0), axis=1).mean()
    assert d_after < 0.25 * d_before, (d_before, d_after)


@pytest.mark.gpu
def test_general_kernel_and_pmg_on_a_scrambled_mesh():
    import torch
    import paper_2205_05136_amd as mf
    from gpu_common import announce, rel_l2, to_dev, to_np
    announce("scrambled mesh apply + p-MG PCG")
    prob, ed, xyz, fib, node_perm, elem_perm, rot = _scrambled(SPEC, 9)
    A = prob.assemble()[0]
    fine = meshops.to_mesh(SPEC.p, ed, xyz, fib)
    op = mf.Operator(fine, sigma_const=SPEC.sigma, alpha=SPEC.alpha, structured=False)
    x = synth.uniform(106, SPEC.n_dof)
    xu = np.empty_like(x)
    xu[node_perm] = x
    yu = to_np(op.apply(to_dev(xu)))
    assert rel_l2(yu[node_perm], A @ x) <= 1e-12
    # p-multigrid on the same elements: the coarse DOF spaces keep each element's
    # rotation and order (their own node numbering), the geometry map stays the fine one
    ops = [op]
    for pc in (1,):
        cprob = oop.Problem(SPEC.with_(p=pc))
        ced = meshops.reorient(cprob.mesh.elem_dof, pc, rot)[elem_perm]
        cperm = np.random.default_rng(10 + pc).permutation(cprob.n_dof)
        coarse = meshops.to_mesh(pc, cperm[ced], np.zeros((cprob.n_dof, 3)), None)
        ops.append(mf.Operator(coarse, geometry=fine, sigma_const=SPEC.sigma, alpha=SPEC.alpha,
                               structured=False))
    mg = mf.Multigrid(ops, [("p",)], degree=3)
    f = synth.uniform(107, SPEC.n_dof)
    fu = np.empty_like(f)
    fu[node_perm] = f
    u, info = mf.pcg(op, to_dev(fu), mg=mg, rtol=1e-13, max_it=100)
    import scipy.sparse.linalg as spla
    u_ref = spla.spsolve(A.tocsc(), f)
    assert rel_l2(to_np(u)[node_perm], u_ref) <= 1e-11
    assert info.iters[0] <= 25
