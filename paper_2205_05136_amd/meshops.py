"""Conforming hexahedral meshes given by arrays instead of the box generator:
element orientation, element and node renumbering, locality ordering, octree
refinement of an arbitrary coarse mesh (the h-levels of the multigrid,
Section 4.3) and the degree-p node maps of its elements (the p-levels).

The operator takes any conforming element-to-node map (Section 3: the Q_p
space on a conforming hexahedral mesh) with the general element kernel
(`Operator(..., structured=False)`): each element's map, Jacobian and fibers
come from its own nodes, so a mesh whose elements are rotated, shuffled and
renumbered gives the same operator up to the permutation of the nodes.  These
helpers build such meshes (from a structured box, for testing and for
reordering real meshes) and a locality order for arbitrary ones.  The
numbering of refined and lower-degree meshes is integer host code; their
node coordinates and fibers are evaluated from the parent map in the library
(mfsem_mesh_refine_nodes, mfsem_mesh_degree_nodes).
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations, product

import numpy as np
import torch


@dataclass
class Mesh:
    """Arrays of a conforming Q_p mesh, usable wherever the operator takes a Box
    (DOF numbering and geometry map of the same degree)."""
    p: int
    elem_dof: torch.Tensor      # [n_elem][(p+1)^3] int32, local index a + P(b + P c)
    xyz: torch.Tensor           # [n_dof][3] float64
    fiber: torch.Tensor | None  # [n_dof][3] float64 or None

    @property
    def n_elem(self):
        return self.elem_dof.shape[0]

    @property
    def n_dof(self):
        return self.xyz.shape[0]

    @property
    def device(self):
        return self.xyz.device

    n = (0, 0, 0)  # not a lattice


def cube_rotations() -> list[np.ndarray]:
    """The 24 proper rotations of the reference cube as signed permutation matrices."""
    out = []
    for perm in permutations(range(3)):
        for signs in product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


def local_rotation_maps(p: int) -> np.ndarray:
    """[24][(p+1)^3]: for each rotation R, the new local index of each old local
    node (a, b, c) when the element's reference axes are rotated by R."""
    P = p + 1
    idx = np.arange(P ** 3)
    a, b, c = idx % P, (idx // P) % P, idx // (P * P)
    s = np.stack([2 * a - p, 2 * b - p, 2 * c - p])  # doubled centred coordinates
    maps = []
    for R in cube_rotations():
        t = (R @ s + p) // 2
        maps.append(t[0] + P * (t[1] + P * t[2]))
    return np.stack(maps)


def reorient(elem_dof: np.ndarray, p: int, rot: np.ndarray) -> np.ndarray:
    """Elements with their local axes rotated: rot[e] in 0..23 per element.
    The element keeps its nodes; only their local order changes."""
    maps = local_rotation_maps(p)
    out = np.empty_like(elem_dof)
    rows = np.arange(elem_dof.shape[0])[:, None]
    out[rows, maps[rot]] = elem_dof
    return out


def permute(mesh_elem_dof: np.ndarray, xyz: np.ndarray, fiber: np.ndarray | None,
            node_perm: np.ndarray, elem_perm: np.ndarray):
    """Renumber nodes (old node g becomes node_perm[g]) and reorder elements
    (new element k is old element elem_perm[k])."""
    ed = node_perm[mesh_elem_dof[elem_perm]]
    xyz_n = np.empty_like(xyz)
    xyz_n[node_perm] = xyz
    fib_n = None
    if fiber is not None:
        fib_n = np.empty_like(fiber)
        fib_n[node_perm] = fiber
    return ed, xyz_n, fib_n


def morton_order(points: np.ndarray, bits: int = 21) -> np.ndarray:
    """Order of points along the Z-order (Morton) curve of their bounding box."""
    lo, hi = points.min(axis=0), points.max(axis=0)
    q = ((points - lo) / np.maximum(hi - lo, 1e-300) * ((1 << bits) - 1)).astype(np.uint64)
    code = np.zeros(len(points), dtype=np.uint64)
    for bit in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + d)
    return np.argsort(code, kind="stable")


def locality_order(elem_dof: np.ndarray, xyz: np.ndarray):
    """Element order along the Morton curve of the element centroids, and a node
    numbering by first appearance in that order: neighbouring elements then share
    nearby node indices, which keeps the gathers and atomics of the general
    element kernel in cache.  Returns (node_perm, elem_perm) for permute()."""
    centroids = xyz[elem_dof].mean(axis=1)
    elem_perm = morton_order(centroids)
    first = np.full(xyz.shape[0], -1, dtype=np.int64)
    order = elem_dof[elem_perm].reshape(-1)
    _, idx = np.unique(order, return_index=True)     # first appearance of each node
    seen = order[np.sort(idx)]
    first[seen] = np.arange(len(seen))
    return first, elem_perm


def to_mesh(p: int, elem_dof: np.ndarray, xyz: np.ndarray, fiber: np.ndarray | None,
            device="cuda") -> Mesh:
    dev = torch.device(device)
    if dev.type == "cuda" and dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    return Mesh(p=p, elem_dof=torch.as_tensor(elem_dof.astype(np.int32), device=dev).contiguous(),
                xyz=torch.as_tensor(xyz, dtype=torch.float64, device=dev).contiguous(),
                fiber=None if fiber is None else
                torch.as_tensor(fiber, dtype=torch.float64, device=dev).contiguous())


# ------------------------------------------------------------------------------
# Node lattices on arbitrary conforming meshes: octree refinement and p-levels.
#
# A node of an element's m-subdivision lattice (local indices I, J, K in 0..m)
# lies in the interior of the element, of one of its faces or edges, or at a
# corner.  Nodes shared by several elements are identified topologically, from
# the global ids of the corners of that face, edge or corner: the anchor is the
# corner with the smallest id, the face's two directions are ordered by the ids
# of the anchor's neighbours along them, and the node's position is its index
# distance from the anchor along each direction.  Every element sharing the
# entity computes the same key (the lattices are symmetric: GLL points and the
# halves of the octree children), so the numbering needs no coordinates.

def element_corners(elem_dof: np.ndarray, p: int) -> np.ndarray:
    """Global ids of each element's 8 corner nodes, [n_elem][8], corner
    (sx, sy, sz) in {0, 1}^3 at column sx + 2 sy + 4 sz."""
    P = p + 1
    cols = [(sx * p) + P * ((sy * p) + P * (sz * p))
            for sz in (0, 1) for sy in (0, 1) for sx in (0, 1)]
    return np.asarray(elem_dof)[:, cols]


def lattice_numbering(corners: np.ndarray, m: int):
    """Global numbering of every element's (m+1)^3 lattice nodes, shared nodes
    identified through the corner ids.  corners [n_elem][8] (element_corners).
    Host preprocessing: it builds a 7-integer key per element node, i.e. about
    56 n_elem (m+1)^3 bytes (1.4 GB for 10^5 elements at m = 6).
    Returns (ids [n_elem][(m+1)^3] with local index I + (m+1)(J + (m+1)K),
    n_nodes, first) where first[g] = (element, local index) of node g's first
    occurrence."""
    corners = np.asarray(corners, dtype=np.int64)
    ne = corners.shape[0]
    M = m + 1
    keys = np.zeros((ne, M ** 3, 7), dtype=np.int64)
    erange = np.arange(ne)
    for K in range(M):
        for J in range(M):
            for I in range(M):
                loc = I + M * (J + M * K)
                idx = (I, J, K)
                side = [0 if v == 0 else (1 if v == m else -1) for v in idx]
                free = [ax for ax in range(3) if side[ax] < 0]
                if len(free) == 3:
                    keys[:, loc, 0] = 3
                    keys[:, loc, 1] = erange
                    keys[:, loc, 2:5] = idx
                    continue
                # corners of the entity: the free axes take both sides
                combos = []
                for bits in range(1 << len(free)):
                    sd = list(side)
                    for k, ax in enumerate(free):
                        sd[ax] = (bits >> k) & 1
                    combos.append(sd[0] + 2 * sd[1] + 4 * sd[2])
                C = corners[:, combos]                          # [ne][2^d]
                amin = np.argmin(C, axis=1)
                v0 = C[erange, amin]
                keys[:, loc, 0] = len(free)
                keys[:, loc, 1] = v0
                if not free:
                    continue
                # the anchor's side on each free axis, its neighbours and distances
                nb, dist = [], []
                for k, ax in enumerate(free):
                    s0 = (amin >> k) & 1                       # anchor side on this axis
                    nb.append(C[erange, amin ^ (1 << k)])
                    dist.append(np.where(s0 == 0, idx[ax], m - idx[ax]))
                if len(free) == 1:
                    keys[:, loc, 2] = nb[0]
                    keys[:, loc, 3] = dist[0]
                else:
                    swap = nb[1] < nb[0]
                    keys[:, loc, 2] = np.where(swap, nb[1], nb[0])
                    keys[:, loc, 3] = np.where(swap, nb[0], nb[1])
                    keys[:, loc, 4] = np.where(swap, dist[1], dist[0])
                    keys[:, loc, 5] = np.where(swap, dist[0], dist[1])
    flat = keys.reshape(-1, 7)
    _, first, inv = np.unique(flat, axis=0, return_index=True, return_inverse=True)
    ids = inv.reshape(ne, M ** 3)
    # number the nodes by first appearance (element order), not by key order
    order = np.argsort(first, kind="stable")
    renum = np.empty_like(order)
    renum[order] = np.arange(len(order))
    ids = renum[ids]
    first = first[order]
    return ids, len(order), np.stack([first // M ** 3, first % M ** 3], axis=1)


def refine_topology(p: int, elem_dof: np.ndarray):
    """The integer part of octree refinement: every element split into its 8
    children and the children's degree-p nodes numbered once across the mesh
    (topologically, lattice_numbering).  Fine element 8 e + c is child
    c = cx + 2 cy + 4 cz of coarse element e, with its local axes those of the
    parent (the convention of the h-transfer).  Returns (elem_dof_fine, parent,
    child, first) with first[g] = (coarse element, point of its (2p+1)^3
    lattice) holding new node g."""
    ed = np.asarray(elem_dof, dtype=np.int64)
    ne, P = ed.shape[0], p + 1
    m = 2 * p
    ids, n_nodes, first = lattice_numbering(element_corners(ed, p), m)
    M = m + 1
    # fine element (e, c) node (a, b, cc) -> lattice (cx p + a, cy p + b, cz p + cc)
    a = np.arange(P)
    A, B, Cc = np.meshgrid(a, a, a, indexing="ij")
    A, B, Cc = (v.transpose(2, 1, 0).reshape(-1) for v in (A, B, Cc))  # local a + P(b + P c)
    fine_ed = np.empty((ne * 8, P ** 3), dtype=np.int64)
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        loc = (cx * p + A) + M * ((cy * p + B) + M * (cz * p + Cc))
        fine_ed[c::8] = ids[:, loc]
    parent = np.repeat(np.arange(ne), 8)
    child = np.tile(np.arange(8), ne)
    return fine_ed, parent, child, first


def degree_topology(p: int, elem_dof: np.ndarray, pc: int):
    """The integer part of a p-level: the degree-pc node map of the same
    elements, nodes numbered once across the mesh.  Returns (elem_dof_pc,
    first) with first[g] = (element, point of its (pc+1)^3 lattice)."""
    ids, n_nodes, first = lattice_numbering(element_corners(np.asarray(elem_dof), p), pc)
    return ids, first


def _place(kind: str, p: int, ed, xyz, fib, first, pc: int = 0, device="cuda"):
    """New node coordinates and fibers from the parent's map, on the device
    (mfsem_mesh_refine_nodes / mfsem_mesh_degree_nodes); returned on the host."""
    from . import api
    dev = torch.device(device)
    t = lambda v, dt: torch.as_tensor(np.ascontiguousarray(v), dtype=dt, device=dev)
    xyz_n, fib_n = api.place_nodes(kind, p, t(ed, torch.int32), t(xyz, torch.float64),
                                   None if fib is None else t(fib, torch.float64),
                                   t(first[:, 0], torch.int32), t(first[:, 1], torch.int32), pc)
    return xyz_n.cpu().numpy(), None if fib_n is None else fib_n.cpu().numpy()


def refine(mesh: "Mesh | tuple", device="cuda"):
    """Octree refinement of a conforming mesh (Section 4.3): the topology of
    refine_topology, and node coordinates and fibers interpolated from the
    parent's map by the library (exact: the parent's degree-p map restricted to
    a child is a degree-p polynomial of the child's reference coordinates).
    Accepts a Mesh or (p, elem_dof, xyz, fiber) numpy arrays.  Returns
    (p, elem_dof, xyz, fiber, parent, child) as numpy arrays."""
    p, ed, xyz, fib = _arrays(mesh)
    fine_ed, parent, child, first = refine_topology(p, ed)
    xyz_f, fib_f = _place("refine", p, ed, xyz, fib, first, device=device)
    return p, fine_ed, xyz_f, fib_f, parent, child


def degree_mesh(mesh: "Mesh | tuple", pc: int, device="cuda"):
    """The degree-pc node map of the same elements (a p-level of the multigrid
    on an arbitrary mesh), nodes numbered once across the mesh and placed by
    the library from the degree-p map.  Returns (pc, elem_dof, xyz, fiber) as
    numpy arrays."""
    p, ed, xyz, fib = _arrays(mesh)
    ids, first = degree_topology(p, ed, pc)
    xyz_c, fib_c = _place("degree", p, ed, xyz, fib, first, pc=pc, device=device)
    return pc, ids, xyz_c, fib_c


def _arrays(mesh):
    if isinstance(mesh, Mesh):
        return (mesh.p, mesh.elem_dof.cpu().numpy().astype(np.int64),
                mesh.xyz.cpu().numpy(), None if mesh.fiber is None else mesh.fiber.cpu().numpy())
    p, ed, xyz, fib = mesh
    return p, np.asarray(ed, dtype=np.int64), np.asarray(xyz, dtype=np.float64), (
        None if fib is None else np.asarray(fib, dtype=np.float64))
