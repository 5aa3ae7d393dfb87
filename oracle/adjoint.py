"""Gradients with respect to per-element conductivities, by explicit matrices.

A(sigma) = alpha M + sum_e P_e^T K_e(sigma_e) P_e is linear in
sigma_e = (sigma_l, sigma_t, sigma_n) of each element, with
dA/dsigma_{e,c} = P_e^T dK_e[c] P_e where dK_e[c] is K_e with the diffusion
tensor replaced by the tensor multiplying sigma_c (f f^T, s s^T, n n^T, or
I - f f^T when no sheet is given; Section 2, the diffusion tensor).

For u = A^{-1} f and L = 1/2 ||u - u_t||^2:
    A lam = u - u_t,   dL/dsigma_{e,c} = -lam^T (dA/dsigma_{e,c}) u,   dL/df = lam.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .operator import Problem


def grad_sigma(prob: Problem, u, w):
    """g[e, c] = w^T (dA/dsigma_{e,c}) u  for every element e and c in (l, t, n)."""
    g = np.zeros((prob.spec.n_elem, 3))
    for el in prob.chunks():
        _, _, dK = prob.elem_matrices(el, parts=True)
        ed = prob.elem_dof[el]
        g[el] = np.einsum("ceij,ei,ej->ec", dK, w[ed], u[ed])
    return g


def solve(prob: Problem, f, A=None):
    if A is None:
        A, _, _ = prob.assemble()
    return spla.spsolve(A.tocsc(), f), A


def loss_and_grad(prob: Problem, f, u_t):
    u, A = solve(prob, f)
    lam = spla.spsolve(A.tocsc(), u - u_t)
    L = 0.5 * float(np.sum((u - u_t) ** 2))
    return L, -grad_sigma(prob, u, lam), lam, u


def loss(prob: Problem, f, u_t):
    u, _ = solve(prob, f)
    return 0.5 * float(np.sum((u - u_t) ** 2))
