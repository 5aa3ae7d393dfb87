"""Conforming hexahedral meshes given by arrays instead of the box generator:
element orientation, element and node renumbering, and locality ordering.

The operator takes any conforming element-to-node map (Section 3: the Q_p
space on a conforming hexahedral mesh) with the general element kernel
(`Operator(..., structured=False)`): each element's map, Jacobian and fibers
come from its own nodes, so a mesh whose elements are rotated, shuffled and
renumbered gives the same operator up to the permutation of the nodes.  These
host-side helpers build such meshes (from a structured box, for testing and
for reordering real meshes) and a locality order for arbitrary ones.
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
