"""The heat-equation BDF1/2/3 study of the paper's appendix, in 3D.

u_t - div(grad u) = f on the unit cube with homogeneous Neumann conditions,
SEM-NI in space (lumped mass M, stiffness K), BDF of order k in time:
    (a0/dt M + K) u^{n+1} = M (f^{n+1} + (1/dt) sum_j a_j u^{n+1-j}).
Two manufactured solutions, as in the appendix:
  "poly":  u = (g(x) + g(y) + g(z)) (2 + sin(pi t)), g(s) = 3 s^2 - 2 s^3, which
           Q_p (p >= 3) reproduces exactly in space (the appendix's x^2 + y^2 is
           replaced by a cubic whose normal derivative vanishes on the faces,
           since the operator carries natural boundary conditions), so the
           error is the time error alone;
  "trig":  u = cos(pi x) cos(pi y) cos(pi z) (2 + sin(pi t)), which is not, so
           the error stops falling at the space error as dt shrinks.
The error is the appendix's discrete L2-in-time norm,
    err = (dt sum_n ||u_h^n - u(t^n)||_M^2)^(1/2),
with the nodal error measured in the mass-matrix norm.  The first k-1 steps
take the exact nodal values.  Test code: the solver callback is the oracle's
direct solve on the CPU or the library's PCG on the GPU.
"""
from __future__ import annotations

import numpy as np

BDF = {1: (1.0, (1.0,)), 2: (1.5, (2.0, -0.5)), 3: (11.0 / 6.0, (3.0, -1.5, 1.0 / 3.0))}


def exact(kind, xyz, t):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    if kind == "poly":
        g = lambda s: 3 * s ** 2 - 2 * s ** 3
        return (g(x) + g(y) + g(z)) * (2 + np.sin(np.pi * t))
    return np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z) * (2 + np.sin(np.pi * t))


def source(kind, xyz, t):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    if kind == "poly":
        g = lambda s: 3 * s ** 2 - 2 * s ** 3
        g2 = lambda s: 6 - 12 * s
        S = g(x) + g(y) + g(z)
        return S * np.pi * np.cos(np.pi * t) - (2 + np.sin(np.pi * t)) * (g2(x) + g2(y) + g2(z))
    U = np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z)
    return U * np.pi * np.cos(np.pi * t) + 3 * np.pi ** 2 * U * (2 + np.sin(np.pi * t))


def run(kind, order, dt, T, xyz, mass, solve):
    """March to T; solve(rhs) returns u^{n+1} of (a0/dt M + K) u = rhs."""
    a0, a = BDF[order]
    n_steps = int(round(T / dt))
    # the first order-1 steps take exact values (hist holds the newest last)
    hist = [exact(kind, xyz, j * dt) for j in range(order)]
    err2 = sum(dt * float(np.sum(mass * (h - exact(kind, xyz, j * dt)) ** 2))
               for j, h in enumerate(hist) if j > 0)
    for n in range(order - 1, n_steps):
        t1 = (n + 1) * dt
        rhs = mass * (source(kind, xyz, t1)
                      + sum(a[j] * hist[-1 - j] for j in range(order)) / dt)
        u = solve(rhs)
        hist = hist[1:] + [u]
        e = u - exact(kind, xyz, t1)
        err2 += dt * float(np.sum(mass * e * e))
    return np.sqrt(err2)
