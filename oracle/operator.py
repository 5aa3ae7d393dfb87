"""The implicit monodomain operator A = alpha*M + K(sigma), by explicit element
matrices (Section 3, the linear system and its matrix A = (3/(2 dt)) M + K, with
the mass coefficient generalised to an input alpha; Section 2, the diffusion
tensor D = sigma_l f f^T + sigma_t s s^T + sigma_n n n^T).

For an element e with isoparametric map X(xi) = sum_i X_i phi_i(xi) and a
quadrature rule {xi_k, W_k} (GLL(p+1) for SEM-NI, Gauss(q) for SEM):

    J_k        = dX/dxi at xi_k,            det J_k > 0 required
    grad phi_i = J_k^{-T} (reference gradient of phi_i)
    M_e[i, j]  = sum_k W_k |J_k| phi_i(xi_k) phi_j(xi_k)
    K_e[i, j]  = sum_k W_k |J_k| (grad phi_i)^T sigma_k (grad phi_j)
    A          = sum_e P_e^T (alpha M_e + K_e) P_e

sigma_k uses the fiber f interpolated to xi_k by the map basis and normalised:
sigma_t I + (sigma_l - sigma_t) f f^T (no sheet), sigma_l f f^T + sigma_t s s^T
+ sigma_n n n^T (sheet s made orthonormal to f, n = f x s), or sigma_t I (no
fiber).  This is the plain definition: element matrices are dense
(P^3 x P^3) and applying them costs O(P^6) per element, with none of the sum
factorisation of Section 4.1.

The DOF space and the geometry may differ in degree: a p-coarsened multigrid
level uses the degree-p_c nodal basis on the same elements while the map stays
the fine isoparametric one.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import basis, mesh as mesh_mod, quadrature


def sigma_tensor(sig_e, f=None, s=None):
    """sigma at a batch of points: sig_e [..., 3] = (sl, st, sn); f, s [..., 3]."""
    sl, st, sn = sig_e[..., 0], sig_e[..., 1], sig_e[..., 2]
    eye = np.eye(3)
    if f is None:
        return st[..., None, None] * eye
    f = f / np.linalg.norm(f, axis=-1, keepdims=True)
    ff = f[..., :, None] * f[..., None, :]
    if s is None:
        return st[..., None, None] * eye + (sl - st)[..., None, None] * ff
    s = s - np.sum(s * f, axis=-1, keepdims=True) * f
    s = s / np.linalg.norm(s, axis=-1, keepdims=True)
    n = np.cross(f, s)
    ss = s[..., :, None] * s[..., None, :]
    nn = n[..., :, None] * n[..., None, :]
    return sl[..., None, None] * ff + st[..., None, None] * ss + sn[..., None, None] * nn


def sigma_parts(f=None, s=None, shape=None):
    """The tensors multiplying sigma_l, sigma_t, sigma_n (dsigma/dsigma_*)."""
    eye = np.eye(3)
    if f is None:
        z = np.zeros(shape + (3, 3))
        return z, np.broadcast_to(eye, shape + (3, 3)).copy(), z
    f = f / np.linalg.norm(f, axis=-1, keepdims=True)
    ff = f[..., :, None] * f[..., None, :]
    if s is None:
        return ff, eye - ff, np.zeros_like(ff)
    s = s - np.sum(s * f, axis=-1, keepdims=True) * f
    s = s / np.linalg.norm(s, axis=-1, keepdims=True)
    n = np.cross(f, s)
    return ff, s[..., :, None] * s[..., None, :], n[..., :, None] * n[..., None, :]


@dataclass
class Geometry:
    """Per element and quadrature point: W|J|, J^{-1}, fiber/sheet at the point."""
    WJ: np.ndarray        # [E, Q^3]
    Jinv: np.ndarray      # [E, Q^3, 3, 3]
    f: np.ndarray | None  # [E, Q^3, 3]
    s: np.ndarray | None


def geometry(Xe, fe, se, map_p, pts, w):
    """Geometry at the tensor quadrature points of a batch of elements.

    Xe [E, Pm^3, 3] map node coordinates; fe/se [E, Pm^3, 3] or None."""
    map_nodes, _ = quadrature.gll(map_p)
    Phi_m, dPhi_m = basis.basis3(map_nodes, pts)
    J = np.einsum("eir,ski->eksr", Xe, dPhi_m).transpose(0, 1, 3, 2)  # J[e,k,r,s] = dX_r/dxi_s
    det = np.linalg.det(J)
    if np.any(det <= 0):
        bad = np.argwhere(det <= 0)[0]
        raise ValueError(f"non-positive Jacobian in element-batch index {bad[0]}, point {bad[1]}")
    W = basis.tensor_weights(w)
    f = None if fe is None else np.einsum("eir,ki->ekr", fe, Phi_m)
    s = None if se is None else np.einsum("eir,ki->ekr", se, Phi_m)
    return Geometry(WJ=W[None, :] * det, Jinv=np.linalg.inv(J), f=f, s=s)


def element_matrices(geo: Geometry, sig_e, dof_p, pts, alpha, parts=False):
    """Dense M_e, K_e [E, P^3, P^3] from the geometry of a batch of elements.

    sig_e [E, 3].  With parts=True also returns dK/dsigma_{l,t,n} [3, E, P^3, P^3]."""
    nodes, _ = quadrature.gll(dof_p)
    Phi, dPhi = basis.basis3(nodes, pts)                      # [Q3, P3], [3, Q3, P3]
    E, Q3 = geo.WJ.shape
    P3 = Phi.shape[1]
    # physical gradients grad[e,k,r,i] = sum_s Jinv[e,k,s,r] dPhi[s,k,i]  (J^{-T} grad_ref)
    grad = np.zeros((E, Q3, 3, P3))
    for s_ in range(3):
        grad += geo.Jinv[:, :, s_, :, None] * dPhi[s_][None, :, None, :]
    # M_e = Phi^T diag(W|J|) Phi
    M = np.matmul(Phi.T[None, :, :] * geo.WJ[:, None, :], Phi[None, :, :])
    sig = sigma_tensor(np.broadcast_to(sig_e[:, None, :], (E, Q3, 3)), geo.f, geo.s)

    def stiffness(T):
        # K_e[i,j] = sum_k sum_r grad[k,r,i] (W|J| T grad)[k,r,j], as one matmul per element
        Tg = np.zeros_like(grad)
        for s_ in range(3):
            Tg += T[:, :, :, s_, None] * grad[:, :, s_, None, :]
        Tg *= geo.WJ[:, :, None, None]
        return np.matmul(grad.reshape(E, 3 * Q3, P3).transpose(0, 2, 1),
                         Tg.reshape(E, 3 * Q3, P3))

    K = stiffness(sig)
    if not parts:
        return M, K
    dK = [stiffness(T) for T in sigma_parts(geo.f, geo.s, (E, Q3))]
    return M, K, np.stack(dK)


class Problem:
    """A discretised operator on a structured box described by a synth.BoxSpec.

    dof_p:  degree of the DOF space (defaults to the mesh degree spec.p);
    quad:   'gll' (SEM-NI, q = dof_p+1) or 'gauss' (SEM, q points);
    sigma:  per-element conductivities [n_elem, 3] or None for spec.sigma;
    jitter: optional per-node displacement [n_dof(spec.p), 3] added to the map
            nodes (keeps det J > 0 when small).
    """

    def __init__(self, spec, dof_p=None, quad=None, q=None, sigma=None, alpha=None,
                 jitter=None, chunk_bytes=256 << 20):
        self.spec = spec
        self.mesh = mesh_mod.box(spec)
        if jitter is not None:
            self.mesh.xyz = self.mesh.xyz + jitter
        self.map_p = spec.p
        self.p = spec.p if dof_p is None else dof_p
        self.quad = quad or spec.quad
        if self.quad == "gll":
            self.q = self.p + 1
        else:
            self.q = q or (spec.q if dof_p is None else self.p + 1)
        self.pts, self.w = quadrature.rule(self.quad, self.p, self.q)
        self.alpha = spec.alpha if alpha is None else alpha
        ne = spec.n_elem
        self.sigma = (np.broadcast_to(np.asarray(spec.sigma, float), (ne, 3)).copy()
                      if sigma is None else np.asarray(sigma, float))
        self.elem_dof = (self.mesh.elem_dof if self.p == spec.p
                         else mesh_mod.elem_dof_map(self.p, spec.n))
        P = self.p + 1
        self.n_dof = int(np.prod([self.p * n + 1 for n in spec.n]))
        per_elem = 8 * (self.q ** 3) * (P ** 3) * 8 + 8 * P ** 6 * 4
        self.chunk = max(1, int(chunk_bytes // per_elem))

    # -- element level ----------------------------------------------------------
    def elem_geometry(self, elems):
        X = self.mesh.xyz[self.mesh.elem_dof[elems]]
        ed = self.mesh.elem_dof[elems]
        f = None if self.mesh.fiber is None else self.mesh.fiber[ed]
        s = None if self.mesh.sheet is None else self.mesh.sheet[ed]
        return geometry(X, f, s, self.map_p, self.pts, self.w)

    def elem_matrices(self, elems, parts=False):
        geo = self.elem_geometry(elems)
        return element_matrices(geo, self.sigma[elems], self.p, self.pts, self.alpha, parts)

    def chunks(self):
        ne = self.spec.n_elem
        for s in range(0, ne, self.chunk):
            yield np.arange(s, min(ne, s + self.chunk))

    # -- R1: assembled sparse matrices (Alg. 2, the matrix-based path) -----------
    def assemble(self):
        """CSR matrices (A, M, K)."""
        P3 = (self.p + 1) ** 3
        rows, cols, vm, vk = [], [], [], []
        for el in self.chunks():
            M, K = self.elem_matrices(el)
            g = self.elem_dof[el]
            rows.append(np.repeat(g, P3, axis=1).reshape(-1))
            cols.append(np.tile(g, (1, P3)).reshape(-1))
            vm.append(M.reshape(-1))
            vk.append(K.reshape(-1))
        rows, cols = np.concatenate(rows), np.concatenate(cols)
        N = self.n_dof
        Mg = sp.csr_matrix((np.concatenate(vm), (rows, cols)), shape=(N, N))
        Kg = sp.csr_matrix((np.concatenate(vk), (rows, cols)), shape=(N, N))
        Mg.sum_duplicates()
        Kg.sum_duplicates()
        A = (self.alpha * Mg + Kg).tocsr()
        return A, Mg, Kg

    # -- R2: dense element action without assembly ------------------------------
    def apply_elementwise(self, x):
        """y = A x as sum_e P_e^T (alpha M_e + K_e) P_e x, element by element."""
        y = np.zeros(self.n_dof)
        for el in self.chunks():
            M, K = self.elem_matrices(el)
            g = self.elem_dof[el]
            ye = np.einsum("eij,ej->ei", self.alpha * M + K, x[g])
            np.add.at(y, g.reshape(-1), ye.reshape(-1))
        return y

    def diagonal(self):
        d = np.zeros(self.n_dof)
        for el in self.chunks():
            M, K = self.elem_matrices(el)
            g = self.elem_dof[el]
            de = np.einsum("eii->ei", self.alpha * M + K)
            np.add.at(d, g.reshape(-1), de.reshape(-1))
        return d


def apply_rows(spec, x_fn, rows, sigma=None):
    """(A x)_g for a few global rows g of a mesh too large to assemble.

    x_fn(global_indices) returns x at those DOFs.  Each row is the sum over the
    (at most 8) elements containing g of row l(g) of alpha*M_e + K_e times x_e.
    Only degree-p GLL/Gauss operators on the spec's own mesh are covered."""
    pts, w = quadrature.rule(spec.quad, spec.p, spec.q)
    out = np.zeros(len(rows))
    for r, g in enumerate(rows):
        elems = mesh_mod.elements_of_dof(spec, int(g))
        xyz, fib, she, gidx = mesh_mod.element_nodes(spec, elems)
        geo = geometry(xyz, fib, she, spec.p, pts, w)
        sig = (np.broadcast_to(np.asarray(spec.sigma, float), (len(elems), 3))
               if sigma is None else sigma[elems])
        M, K = element_matrices(geo, sig, spec.p, pts, spec.alpha)
        for i in range(len(elems)):
            l = int(np.nonzero(gidx[i] == g)[0][0])
            out[r] += (spec.alpha * M[i, l] + K[i, l]) @ x_fn(gidx[i])
    return out
