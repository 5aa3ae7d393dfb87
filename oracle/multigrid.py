"""Inter-level transfers and the level hierarchy of the geometric multigrid
preconditioner (Section 4.3: high-order h-multigrid with p-degree
interpolation and restriction among octree meshes refined from a coarse mesh).

Prolongation is interpolation: P[i, j] = phi^c_j(x^f_i), the coarse nodal basis
function j evaluated at fine node i, where the fine node's reference
coordinate inside the coarse element is
  * the same reference coordinate (p-coarsening, same elements);
  * (xi_f + 2c - 1)/2 per axis for child offset c in {0, 1} (octree
    coarsening, parent element = child index // 2).
Restriction is the exact transpose P^T.  Matrices are explicit sparse.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis, mesh as mesh_mod, quadrature


def _first_owner(elem_dof, n_dof):
    """For each global DOF, one (element, local index) containing it."""
    flat = elem_dof.reshape(-1)
    _, first = np.unique(flat, return_index=True)
    P3 = elem_dof.shape[1]
    return first // P3, first % P3


def prolongation_p(n, p_fine, p_coarse):
    """P for p-coarsening on an nx x ny x nz box: [N_f, N_c]."""
    ed_f = mesh_mod.elem_dof_map(p_fine, n)
    ed_c = mesh_mod.elem_dof_map(p_coarse, n)
    N_f = int(np.prod([p_fine * k + 1 for k in n]))
    N_c = int(np.prod([p_coarse * k + 1 for k in n]))
    xf, _ = quadrature.gll(p_fine)
    xc, _ = quadrature.gll(p_coarse)
    I1 = basis.lagrange(xc, xf)                     # [Pf, Pc]
    I3 = basis.tensor3(I1, I1, I1)                  # [Pf^3, Pc^3]
    e, l = _first_owner(ed_f, N_f)
    g_f = ed_f[e, l]
    rows = np.repeat(g_f, I3.shape[1])
    cols = ed_c[e].reshape(-1)
    vals = I3[l].reshape(-1)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(N_f, N_c))
    P.eliminate_zeros()
    return P


def prolongation_h(n_fine, p):
    """P for octree coarsening n -> n/2 per axis at fixed degree p: [N_f, N_c]."""
    nx, ny, nz = n_fine
    if nx % 2 or ny % 2 or nz % 2:
        raise ValueError("octree coarsening needs even element counts")
    n_c = (nx // 2, ny // 2, nz // 2)
    ed_f = mesh_mod.elem_dof_map(p, n_fine)
    ed_c = mesh_mod.elem_dof_map(p, n_c)
    N_f = int(np.prod([p * k + 1 for k in n_fine]))
    N_c = int(np.prod([p * k + 1 for k in n_c]))
    x, _ = quadrature.gll(p)
    half = [basis.lagrange(x, (x + 2 * c - 1) / 2.0) for c in (0, 1)]  # [P, P] per child
    e, l = _first_owner(ed_f, N_f)
    ex, rem = e % nx, e // nx
    ey, ez = rem % ny, rem // ny
    parent = ex // 2 + n_c[0] * (ey // 2 + n_c[1] * (ez // 2))
    P1 = p + 1
    a, b, c = l % P1, (l // P1) % P1, l // (P1 * P1)
    rows, cols, vals = [], [], []
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                I3 = basis.tensor3(half[cx], half[cy], half[cz])
                m = (ex % 2 == cx) & (ey % 2 == cy) & (ez % 2 == cz)
                g = ed_f[e[m], l[m]]
                rows.append(np.repeat(g, I3.shape[1]))
                cols.append(ed_c[parent[m]].reshape(-1))
                vals.append(I3[l[m]].reshape(-1))
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N_f, N_c))
    P.eliminate_zeros()
    return P
