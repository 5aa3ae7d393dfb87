"""1D quadrature rules on [-1, 1] (Section 3, the SEM and SEM-NI paragraphs).

* Legendre-Gauss (LG) with q points, exact for polynomials of degree 2q-1;
  SEM uses it, typically with p+1 points.
* Legendre-Gauss-Lobatto (LGL/GLL) with p+1 points: the two end points plus the
  roots of P_p'; exact for degree 2p-1.  The same points are the support nodes
  of the nodal Lagrange basis, which makes the SEM-NI mass matrix diagonal.

Both are computed from the Legendre three-term recurrence and Newton's method.
"""
from __future__ import annotations

import numpy as np


def legendre(n: int, x):
    """P_n(x) and P_n'(x) by the recurrence (k+1)P_{k+1} = (2k+1)xP_k - kP_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    d0, d1 = np.zeros_like(x), np.ones_like(x)
    for k in range(1, n):
        p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
        # derivative of the recurrence: P'_{k+1} = P'_{k-1} + (2k+1) P_k
        d2 = d0 + (2 * k + 1) * p1
        p0, p1, d0, d1 = p1, p2, d1, d2
    return p1, d1


def gauss(q: int):
    """Legendre-Gauss points (roots of P_q) and weights 2/((1-x^2) P_q'(x)^2)."""
    if q < 1:
        raise ValueError("q >= 1")
    i = np.arange(q)
    x = -np.cos(np.pi * (i + 0.75) / (q + 0.5))  # ascending initial guesses
    for _ in range(100):
        p, dp = legendre(q, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    _, dp = legendre(q, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    return x, w


def gll(p: int):
    """Gauss-Legendre-Lobatto points and weights, p+1 of them (p >= 1).

    Interior points are the roots of P_p', found by Newton with the second
    derivative taken from Legendre's equation
    (1 - x^2) P'' = 2x P' - p(p+1) P.  Weights are 2 / (p(p+1) P_p(x)^2).
    """
    if p < 1:
        raise ValueError("p >= 1")
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    x[0], x[-1] = -1.0, 1.0
    if p > 1:
        xi = x[1:-1].copy()
        for _ in range(100):
            P, dP = legendre(p, xi)
            d2P = (2 * xi * dP - p * (p + 1) * P) / (1.0 - xi * xi)
            dx = dP / d2P
            xi = xi - dx
            if np.max(np.abs(dx)) < 1e-16:
                break
        x[1:-1] = xi
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P * P)
    return x, w


def rule(kind: str, p: int, q: int | None = None):
    """The quadrature used by a degree-p discretisation: GLL(p+1) or Gauss(q)."""
    if kind == "gll":
        if q not in (None, p + 1):
            raise ValueError("GLL quadrature has exactly p+1 points")
        return gll(p)
    if kind == "gauss":
        return gauss(q if q else p + 1)
    raise ValueError(kind)
