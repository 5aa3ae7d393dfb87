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


# ------------------------------------------------------- refinement / p-levels
# An unsheared box with a uniform fiber: its geometry and fibers are polynomial,
# so the refined mesh is exactly the box at twice the elements.
BOX = synth.BoxSpec(p=3, n=(2, 2, 1), length=(2.0, 1.6, 1.0), fiber=True, theta0=0.6,
                    theta1=0.6, sigma=(0.17, 0.05, 0.05), alpha=3.0)


def _struct_elem(spec, ex, ey, ez):
    return ex + spec.n[0] * (ey + spec.n[1] * ez)


def test_lattice_numbering_counts_on_a_box():
    from oracle import mesh as omesh
    m = omesh.box(BOX)
    for sub in (1, 2, 3, 6):
        ids, n, first = meshops.lattice_numbering(meshops.element_corners(m.elem_dof, BOX.p), sub)
        assert n == np.prod([sub * k + 1 for k in BOX.n])
        assert ids.max() == n - 1 and np.array_equal(np.unique(ids), np.arange(n))
        # the first occurrence of node g is an element that holds it there
        assert np.array_equal(ids[first[:, 0], first[:, 1]], np.arange(n))


def _bijective(a, b):
    """a[k] <-> b[k] pairs define one bijection between the two node sets."""
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    pairs = np.unique(np.stack([a, b], axis=1), axis=0)
    return (len(pairs) == len(np.unique(a)) == len(np.unique(b)))


def test_refine_topology_is_the_box_at_twice_the_elements():
    """Refining a box numbers the children's nodes like the box at twice the
    elements, up to a renumbering (integer part, no coordinates): the fine
    element maps pair with the fine box's maps one to one."""
    from oracle import mesh as omesh
    m = omesh.box(BOX)
    ed, parent, child, first = meshops.refine_topology(BOX.p, m.elem_dof)
    fine = BOX.with_(n=tuple(2 * k for k in BOX.n))
    mf_ = omesh.box(fine)
    assert ed.shape == (fine.n_elem, (BOX.p + 1) ** 3) and ed.max() + 1 == fine.n_dof
    s_of = np.empty(fine.n_elem, dtype=np.int64)
    for e in range(BOX.n_elem):
        ex, ey, ez = e % BOX.n[0], (e // BOX.n[0]) % BOX.n[1], e // (BOX.n[0] * BOX.n[1])
        for c in range(8):
            f = 8 * e + c
            assert parent[f] == e and child[f] == c
            s_of[f] = _struct_elem(fine, 2 * ex + (c & 1), 2 * ey + ((c >> 1) & 1), 2 * ez + (c >> 2))
    assert _bijective(ed, mf_.elem_dof[s_of])
    # the recorded first occurrence of each node is a lattice point of its element
    assert np.all((first[:, 1] >= 0) & (first[:, 1] < (2 * BOX.p + 1) ** 3))


def test_degree_topology_is_the_lower_degree_box():
    from oracle import mesh as omesh
    ced, cxyz, cfib = _scrambled_coarse(BOX, 12)
    for pc in (1, 2, 3):
        ids, first = meshops.degree_topology(BOX.p, ced, pc)
        assert ids.max() + 1 == omesh.box(BOX.with_(p=pc)).xyz.shape[0]
        assert np.array_equal(np.unique(ids), np.arange(ids.max() + 1))
        # corners keep the coarse mesh's corner identity
        assert _bijective(meshops.element_corners(ids, pc), meshops.element_corners(ced, BOX.p))


@pytest.mark.gpu
def test_refined_box_is_the_box_at_twice_the_elements():
    from oracle import mesh as omesh
    m = omesh.box(BOX)
    p, ed, xyz, fib, parent, child = meshops.refine((BOX.p, m.elem_dof, m.xyz, m.fiber))
    fine = BOX.with_(n=tuple(2 * k for k in BOX.n))
    mf_ = omesh.box(fine)
    assert xyz.shape[0] == fine.n_dof and ed.shape[0] == fine.n_elem
    for e in range(BOX.n_elem):
        ex, ey, ez = e % BOX.n[0], (e // BOX.n[0]) % BOX.n[1], e // (BOX.n[0] * BOX.n[1])
        for c in range(8):
            f = 8 * e + c
            assert parent[f] == e and child[f] == c
            s = _struct_elem(fine, 2 * ex + (c & 1), 2 * ey + ((c >> 1) & 1), 2 * ez + (c >> 2))
            np.testing.assert_allclose(xyz[ed[f]], mf_.xyz[mf_.elem_dof[s]], atol=1e-14)
            np.testing.assert_allclose(fib[ed[f]], mf_.fiber[mf_.elem_dof[s]], atol=1e-14)


def _scrambled_coarse(spec, seed):
    from oracle import mesh as omesh
    m = omesh.box(spec)
    rng = np.random.default_rng(seed)
    rot = rng.integers(0, 24, spec.n_elem)
    ed = meshops.reorient(m.elem_dof, spec.p, rot)
    return meshops.permute(ed, m.xyz, m.fiber, rng.permutation(spec.n_dof),
                           rng.permutation(spec.n_elem))


def _match(xyz_a, xyz_b):
    """perm with xyz_a[perm] == xyz_b (nodes matched by coordinates)."""
    ka = np.round(xyz_a / 1e-9).astype(np.int64)
    kb = np.round(xyz_b / 1e-9).astype(np.int64)
    ia = np.lexsort(ka.T[::-1])
    ib = np.lexsort(kb.T[::-1])
    assert np.array_equal(ka[ia], kb[ib])
    perm = np.empty(len(ib), dtype=np.int64)
    perm[ib] = ia
    return perm


def _h_prolongation(p, ed_f, ed_c, parent, child, n_f, n_c):
    """Element-wise interpolation from each parent at its child's nodes."""
    from oracle import basis, quadrature
    x, _ = quadrature.gll(p)
    half = [basis.lagrange(x, (x + 2 * c - 1) / 2.0) for c in (0, 1)]
    Pm = np.zeros((n_f, n_c))
    for f in range(ed_f.shape[0]):
        c = child[f]
        I3 = basis.tensor3(half[c & 1], half[(c >> 1) & 1], half[(c >> 2) & 1])
        Pm[np.ix_(ed_f[f], ed_c[parent[f]])] = I3
    return Pm


@pytest.mark.gpu
def test_refined_scrambled_mesh_operator_and_h_prolongation():
    """Refining a rotated, shuffled, renumbered coarse box gives the permuted
    operator of the box at twice the elements, and its parent/child maps give
    the permuted octree prolongation."""
    from oracle import multigrid as omg
    ced, cxyz, cfib = _scrambled_coarse(BOX, 11)
    p, ed, xyz, fib, parent, child = meshops.refine((BOX.p, ced, cxyz, cfib))
    fine = BOX.with_(n=tuple(2 * k for k in BOX.n))
    prob = oop.Problem(fine)
    A = prob.assemble()[0]
    pf = _match(xyz, prob.mesh.xyz)            # xyz[pf] = structured node order
    Au = _assemble(prob, fine, ed, xyz, fib, np.broadcast_to(prob.sigma[0], (fine.n_elem, 3)))
    Pf = sp.csr_matrix((np.ones(fine.n_dof), (pf, np.arange(fine.n_dof))), shape=(fine.n_dof,) * 2)
    assert abs(Au - Pf @ A @ Pf.T).max() <= 1e-13 * abs(A).max()
    from oracle import mesh as omesh
    pc = _match(cxyz, omesh.box(BOX).xyz)
    Pu = _h_prolongation(p, ed, ced, parent, child, fine.n_dof, BOX.n_dof)
    Ps = omg.prolongation_h(fine.n, p).toarray()
    np.testing.assert_allclose(Pu[np.ix_(pf, pc)], Ps, atol=1e-14)


@pytest.mark.gpu
def test_degree_mesh_is_the_lower_degree_box():
    from oracle import mesh as omesh
    ced, cxyz, cfib = _scrambled_coarse(BOX, 12)
    for pc in (1, 2):
        q, ed, xyz, fib = meshops.degree_mesh((BOX.p, ced, cxyz, cfib), pc)
        box_c = omesh.box(BOX.with_(p=pc))
        assert xyz.shape[0] == box_c.xyz.shape[0]
        _match(xyz, box_c.xyz)
        # each element's degree-pc nodes sit at its degree-p map's GLL(pc) points
        assert np.array_equal(np.unique(ed), np.arange(xyz.shape[0]))
        corners_p = meshops.element_corners(ced, BOX.p)
        corners_c = meshops.element_corners(ed, pc)
        np.testing.assert_allclose(cxyz[corners_p], xyz[corners_c], atol=1e-14)


@pytest.mark.gpu
def test_hp_multigrid_on_a_refined_scrambled_mesh():
    """Octree h-level and p-level built from arrays (refine, degree_mesh) on an
    unstructured mesh: the h-prolongation equals the permuted oracle's and the
    h+p multigrid PCG solves the permuted oracle system."""
    import torch
    import paper_2205_05136_amd as mf
    from gpu_common import announce, rel_l2, to_dev, to_np
    from oracle import mesh as omesh
    from oracle import multigrid as omg
    import scipy.sparse.linalg as spla
    announce("refined scrambled mesh h+p multigrid")
    spec = BOX.with_(n=(4, 2, 2))
    ced, cxyz, cfib = _scrambled_coarse(spec, 13)
    p, ed, xyz, fib, parent, child = meshops.refine((spec.p, ced, cxyz, cfib))
    fine = spec.with_(n=tuple(2 * k for k in spec.n))
    prob = oop.Problem(fine)
    A = prob.assemble()[0]
    pf = _match(xyz, prob.mesh.xyz)
    pc = _match(cxyz, omesh.box(spec).xyz)
    kw = dict(sigma_const=spec.sigma, alpha=spec.alpha, structured=False)
    m_f = meshops.to_mesh(p, ed, xyz, fib)
    m_c = meshops.to_mesh(p, ced, cxyz, cfib)
    q, ed1, xyz1, fib1 = meshops.degree_mesh((spec.p, ced, cxyz, cfib), 1)
    m_1 = meshops.to_mesh(1, ed1, xyz1, fib1)
    ops = [mf.Operator(m_f, **kw), mf.Operator(m_c, **kw), mf.Operator(m_1, geometry=m_c, **kw)]
    par = torch.as_tensor(parent.astype(np.int32), device="cuda")
    chi = torch.as_tensor(child.astype(np.int8), device="cuda")
    mg = mf.Multigrid(ops, [("h", par, chi), ("p",)], degree=3)
    # h-prolongation against the oracle's, permuted
    Ps = omg.prolongation_h(fine.n, p)
    xc = synth.uniform(120, spec.n_dof)
    xcu = np.empty_like(xc)
    xcu[pc] = xc
    yu = to_np(mg.prolong(0, to_dev(xcu)))
    assert rel_l2(yu[pf], Ps @ xc) <= 1e-12
    # the fine operator and the solve
    x = synth.uniform(121, fine.n_dof)
    xu = np.empty_like(x)
    xu[pf] = x
    assert rel_l2(to_np(ops[0].apply(to_dev(xu)))[pf], A @ x) <= 1e-12
    f = synth.uniform(122, fine.n_dof)
    fu = np.empty_like(f)
    fu[pf] = f
    u, info = mf.pcg(ops[0], to_dev(fu), mg=mg, rtol=1e-12, max_it=100)
    u_ref = spla.spsolve(A.tocsc(), f)
    assert rel_l2(to_np(u)[pf], u_ref) <= 1e-10
    assert info.iters[0] <= 20, info.iters


@pytest.mark.parametrize("seed", range(6))
def test_refine_topology_on_random_scrambled_boxes(seed):
    """Random box sizes, degrees and scramblings: the refined and degree-pc
    numberings have the structured node counts (integer part)."""
    rng = np.random.default_rng(100 + seed)
    p = int(rng.integers(1, 5))
    n = tuple(int(v) for v in rng.integers(1, 4, 3))
    spec = synth.BoxSpec(p=p, n=n, length=tuple(rng.uniform(0.5, 2.0, 3)), fiber=True,
                         theta0=0.3, theta1=0.3)
    ced, cxyz, cfib = _scrambled_coarse(spec, 200 + seed)
    ed, parent, child, first = meshops.refine_topology(p, ced)
    assert ed.max() + 1 == np.prod([2 * p * k + 1 for k in n]) and ed.shape[0] == 8 * spec.n_elem
    pc = int(rng.integers(1, p + 1))
    ids, _ = meshops.degree_topology(p, ced, pc)
    assert ids.max() + 1 == np.prod([pc * k + 1 for k in n])


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(6))
def test_refine_and_degree_mesh_on_random_scrambled_boxes(seed):
    """Random box sizes, degrees and scramblings: the refined mesh and the
    degree-pc mesh have the structured node counts and node positions."""
    from oracle import mesh as omesh
    rng = np.random.default_rng(100 + seed)
    p = int(rng.integers(1, 5))
    n = tuple(int(v) for v in rng.integers(1, 4, 3))
    spec = synth.BoxSpec(p=p, n=n, length=tuple(rng.uniform(0.5, 2.0, 3)), fiber=True,
                         theta0=0.3, theta1=0.3)
    ced, cxyz, cfib = _scrambled_coarse(spec, 200 + seed)
    q, ed, xyz, fib, parent, child = meshops.refine((p, ced, cxyz, cfib))
    fine = omesh.box(spec.with_(n=tuple(2 * k for k in n)))
    assert xyz.shape[0] == fine.xyz.shape[0] and ed.shape[0] == 8 * spec.n_elem
    _match(xyz, fine.xyz)
    # every fine element's nodes lie inside its parent's bounding box
    lo = cxyz[ced].min(axis=1)[parent] - 1e-12
    hi = cxyz[ced].max(axis=1)[parent] + 1e-12
    assert np.all((xyz[ed] >= lo[:, None, :]) & (xyz[ed] <= hi[:, None, :]))
    pc = int(rng.integers(1, p + 1))
    _, ed_c, xyz_c, _ = meshops.degree_mesh((p, ced, cxyz, cfib), pc)
    _match(xyz_c, omesh.box(spec.with_(p=pc)).xyz)


@pytest.mark.gpu
def test_place_nodes_argument_and_range_errors():
    """Node placement through the C ABI: a bad degree or lattice is refused on
    the host (EINVAL), and an element or lattice index out of range gives NaN
    coordinates for that node only (the kernel reads nothing out of bounds)."""
    import torch
    import paper_2205_05136_amd as mf
    from paper_2205_05136_amd import api
    from gpu_common import announce
    from oracle import mesh as omesh
    announce("place nodes: errors")
    m = omesh.box(BOX)
    t = lambda v, dt: torch.as_tensor(np.ascontiguousarray(v), dtype=dt, device="cuda")
    ed, xyz = t(m.elem_dof, torch.int32), t(m.xyz, torch.float64)
    elem = t([0, BOX.n_elem, -1, 1], torch.int32)
    loc = t([0, 0, 0, (2 * BOX.p + 1) ** 3], torch.int32)
    out, _ = api.place_nodes("refine", BOX.p, ed, xyz, None, elem, loc)
    o = out.cpu().numpy()
    np.testing.assert_allclose(o[0], m.xyz[m.elem_dof[0, 0]], atol=1e-14)
    assert np.isnan(o[1:]).all()
    with pytest.raises(mf.MfsemError):
        api.place_nodes("degree", BOX.p, ed, xyz, None, elem, loc, pc=0)
    with pytest.raises(mf.MfsemError):
        api.place_nodes("refine", 0, ed, xyz, None, elem, loc)
