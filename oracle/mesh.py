"""Structured hexahedral meshes of degree p (Section 3: conforming hexahedral
meshes and the global space V_{h,p} of continuous piecewise Q_p functions).

Global node (I, J, K) of the (p*nx+1) x (p*ny+1) x (p*nz+1) lattice has index
g = I + NX*(J + NY*K).  Element (ex, ey, ez) has index e = ex + nx*(ey + ny*ez)
and local node (a, b, c) -> global (p*ex + a, p*ey + b, p*ez + c).  Inside an
element the nodes sit at the GLL points mapped to the element; the geometry is
the isoparametric Q_p map through all element nodes.

The recipe (shear, fiber) is the one stated by `synth.BoxSpec`.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .quadrature import gll


@dataclass
class Mesh:
    p: int
    n: tuple
    xyz: np.ndarray        # [n_dof, 3]
    elem_dof: np.ndarray   # [n_elem, P^3] int64
    fiber: np.ndarray | None  # [n_dof, 3] or None
    sheet: np.ndarray | None = None  # [n_dof, 3] or None

    @property
    def n_dof(self):
        return self.xyz.shape[0]

    @property
    def n_elem(self):
        return self.elem_dof.shape[0]


def lattice_1d(p: int, n: int, x0: float, L: float):
    """Node coordinates along one axis: n elements of length L/n, GLL inside."""
    xi, _ = gll(p)
    h = L / n
    out = np.empty(p * n + 1)
    for e in range(n):
        for a in range(p + 1):
            out[p * e + a] = x0 + h * (e + 0.5 * (xi[a] + 1.0))
    return out


def elem_dof_map(p: int, n: tuple):
    nx, ny, nz = n
    NX, NY = p * nx + 1, p * ny + 1
    P = p + 1
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ex, ey, ez = (v.transpose(2, 1, 0).reshape(-1) for v in (ex, ey, ez))  # e = ex + nx(ey + ny ez)
    a = np.arange(P)
    A, B, C = np.meshgrid(a, a, a, indexing="ij")
    A, B, C = (v.transpose(2, 1, 0).reshape(-1) for v in (A, B, C))         # i = a + P(b + P c)
    I = p * ex[:, None] + A[None, :]
    J = p * ey[:, None] + B[None, :]
    K = p * ez[:, None] + C[None, :]
    return (I + NX * (J + NY * K)).astype(np.int64)


def box(spec) -> Mesh:
    """Build the mesh a `synth.BoxSpec` describes."""
    p, (nx, ny, nz) = spec.p, spec.n
    gx = lattice_1d(p, nx, spec.origin[0], spec.length[0])
    gy = lattice_1d(p, ny, spec.origin[1], spec.length[1])
    gz = lattice_1d(p, nz, spec.origin[2], spec.length[2])
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    xyz = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    fiber = sheet = None
    if spec.fiber:
        t = (xyz[:, 2] - spec.origin[2]) / spec.length[2]
        theta = spec.theta0 + (spec.theta1 - spec.theta0) * t
        fiber = np.stack([np.cos(theta), np.sin(theta), np.zeros_like(theta)], axis=1)
        if spec.sheet:
            sheet = np.stack([-np.sin(theta), np.cos(theta), np.zeros_like(theta)], axis=1)
    if spec.shear_amp != 0.0:
        hx = spec.length[0] / nx
        d = spec.shear_amp * hx * np.sin(2 * np.pi * (xyz[:, 0] - spec.origin[0]) / spec.length[0])
        xyz = xyz + d[:, None]
    return Mesh(p=p, n=(nx, ny, nz), xyz=xyz, elem_dof=elem_dof_map(p, (nx, ny, nz)), fiber=fiber,
                sheet=sheet)


def element_ids(n: tuple):
    nx, ny, nz = n
    return np.arange(nx * ny * nz)


def element_nodes(spec, elems):
    """Node coordinates [len(elems), P^3, 3] and fibers of selected elements,
    computed from the recipe without building the global lattice (for meshes
    too large to hold in full)."""
    p, (nx, ny, nz) = spec.p, spec.n
    P = p + 1
    xi, _ = gll(p)
    elems = np.asarray(elems, dtype=np.int64)
    ex, rem = elems % nx, elems // nx
    ey, ez = rem % ny, rem // ny
    hx, hy, hz = (spec.length[i] / spec.n[i] for i in range(3))
    a = np.arange(P)
    A, B, C = np.meshgrid(a, a, a, indexing="ij")
    A, B, C = (v.transpose(2, 1, 0).reshape(-1) for v in (A, B, C))
    x = spec.origin[0] + hx * (ex[:, None] + 0.5 * (xi[A][None, :] + 1.0))
    y = spec.origin[1] + hy * (ey[:, None] + 0.5 * (xi[B][None, :] + 1.0))
    z = spec.origin[2] + hz * (ez[:, None] + 0.5 * (xi[C][None, :] + 1.0))
    xyz = np.stack([x, y, z], axis=-1)
    fib = she = None
    if spec.fiber:
        theta = spec.theta0 + (spec.theta1 - spec.theta0) * (z - spec.origin[2]) / spec.length[2]
        fib = np.stack([np.cos(theta), np.sin(theta), np.zeros_like(theta)], axis=-1)
        if spec.sheet:
            she = np.stack([-np.sin(theta), np.cos(theta), np.zeros_like(theta)], axis=-1)
    if spec.shear_amp != 0.0:
        d = spec.shear_amp * hx * np.sin(2 * np.pi * (x - spec.origin[0]) / spec.length[0])
        xyz = xyz + d[..., None]
    NX, NY = p * nx + 1, p * ny + 1
    gidx = (p * ex[:, None] + A) + NX * ((p * ey[:, None] + B) + NY * (p * ez[:, None] + C))
    return xyz, fib, she, gidx


def elements_of_dof(spec, g):
    """All elements that contain global node g (1 to 8 of them)."""
    p, (nx, ny, nz) = spec.p, spec.n
    NX, NY = p * nx + 1, p * ny + 1
    I, r = g % NX, g // NX
    J, K = r % NY, r // NY

    def cand(i, n):
        e = i // p
        out = []
        if i % p == 0 and e > 0:
            out.append(e - 1)
        if e < n:
            out.append(e)
        return out

    res = []
    for ez in cand(K, nz):
        for ey in cand(J, ny):
            for ex in cand(I, nx):
                res.append(ex + nx * (ey + ny * ez))
    return res
