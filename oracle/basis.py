"""Nodal Lagrange bases on the GLL support nodes (Section 3: the SEM basis is
the tensor product of univariate Lagrange polynomials whose nodes are the LGL
points mapped to each element).

Everything is built from the product formula
    l_a(x) = prod_{m != a} (x - x_m) / (x_a - x_m)
and its derivative, evaluated point by point.  The 3D basis is formed
explicitly as dense (points x basis) arrays: no sum factorisation is used
anywhere in the oracle.

Local numbering: basis index i = a + P*(b + P*c) with P = p+1 (x fastest);
point index k = k1 + Q*(k2 + Q*k3) for a tensor point set of Q per axis.
"""
from __future__ import annotations

import numpy as np


def lagrange(nodes, x):
    """L[k, a] = l_a(x_k)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    P = len(nodes)
    L = np.ones((len(x), P))
    for a in range(P):
        for m in range(P):
            if m != a:
                L[:, a] *= (x - nodes[m]) / (nodes[a] - nodes[m])
    return L


def lagrange_deriv(nodes, x):
    """D[k, a] = l_a'(x_k) = sum_{m != a} 1/(x_a - x_m) prod_{n != a, m} (x - x_n)/(x_a - x_n)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    P = len(nodes)
    D = np.zeros((len(x), P))
    for a in range(P):
        for m in range(P):
            if m == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[m]))
            for n in range(P):
                if n != a and n != m:
                    term *= (x - nodes[n]) / (nodes[a] - nodes[n])
            D[:, a] += term
    return D


def tensor3(A1, A2, A3):
    """Dense 3D array T[k, i] = A1[k1,a] A2[k2,b] A3[k3,c] with
    k = k1 + Q(k2 + Q k3), i = a + P(b + P c)."""
    T = np.einsum("xa,yb,zc->zyxcba", A1, A2, A3)
    Q = A1.shape[0]
    P = A1.shape[1]
    return T.reshape(Q ** 3, P ** 3)


def basis3(nodes, pts):
    """Phi [Q^3, P^3] and reference gradients dPhi [3, Q^3, P^3] of the 3D nodal
    basis on `nodes` (per axis) at the tensor point set `pts` (per axis)."""
    B = lagrange(nodes, pts)
    D = lagrange_deriv(nodes, pts)
    Phi = tensor3(B, B, B)
    dPhi = np.stack([tensor3(D, B, B), tensor3(B, D, B), tensor3(B, B, D)])
    return Phi, dPhi


def tensor_weights(w):
    """W[k] = w[k1] w[k2] w[k3]."""
    return np.einsum("z,y,x->zyx", w, w, w).reshape(-1)
