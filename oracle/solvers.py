"""Linear solvers of Section 4 (CG/PCG for the SPD system A u = b) and the
multigrid ingredients of Section 4.3 (Chebyshev-Jacobi smoother whose range
comes from a CG/Lanczos eigenvalue estimate; Section 5 fixes 10 CG
sub-iterations and the range [0.08, 1.2] * lambda_max), written on explicit
matrices.  Also a textbook fast-diagonalisation solve for tensor-product boxes,
used to pin the assembled operator.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def cg(A, b, x0=None, rtol=1e-10, atol=0.0, max_it=100000, M=None, flexible=False):
    """(P)CG.  Stops when ||r||_2 <= max(rtol*||b||_2, atol).  M(r) applies the
    preconditioner.  flexible=True uses the Polak-Ribiere beta
    (r_{k+1}, z_{k+1} - z_k) / (r_k, z_k).  Returns (x, iterations, ||r||)."""
    Amul = (lambda v: A @ v) if not callable(A) else A
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - Amul(x) if x0 is not None else b.copy()
    tol = max(rtol * np.linalg.norm(b), atol)
    rn = np.linalg.norm(r)
    if rn <= tol:
        return x, 0, rn
    z = M(r) if M else r.copy()
    p = z.copy()
    rz = r @ z
    for it in range(1, max_it + 1):
        q = Amul(p)
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        rn = np.linalg.norm(r)
        if rn <= tol:
            return x, it, rn
        z_old = z
        z = M(r) if M else r.copy()
        rz_new = r @ z
        beta = ((rz_new - r @ z_old) if flexible else rz_new) / rz
        rz = rz_new
        p = z + beta * p
    return x, max_it, rn


def lanczos_lambda_max(A, dinv, v0, iters=10):
    """Largest eigenvalue estimate of D^{-1} A from `iters` Jacobi-PCG steps on
    A x = v0 (x0 = 0): the Lanczos tridiagonal built from the CG coefficients,
    T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_{j,j+1} = sqrt(b_j)/a_j."""
    Amul = (lambda v: A @ v) if not callable(A) else A
    r = v0.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(iters):
        q = Amul(p)
        a = rz / (p @ q)
        r = r - a * q
        z = dinv * r
        rz_new = r @ z
        bta = rz_new / rz
        alphas.append(a)
        betas.append(bta)
        rz = rz_new
        p = z + bta * p
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return float(np.max(np.linalg.eigvalsh(T)))


def chebyshev(A, dinv, b, x0, lam_max, degree, lo=0.08, hi=1.2):
    """Chebyshev-Jacobi smoothing of A x = b on [lo, hi] * lam_max.

    theta = (l_hi + l_lo)/2, delta = (l_hi - l_lo)/2, s = theta/delta, rho = 1/s.
    r = b - A x0 (skipped, r = b, when x0 is None); d = D^{-1} r / theta; x = x0 + d;
    then for j = 2..degree: r = b - A x; rho' = 1/(2s - rho);
    d = rho' rho d + (2 rho'/delta) D^{-1} r; x += d; rho = rho'.
    With x0 given this costs `degree` matrix-vector products, with x0 = None one fewer."""
    Amul = (lambda v: A @ v) if not callable(A) else A
    l_lo, l_hi = lo * lam_max, hi * lam_max
    theta, delta = 0.5 * (l_hi + l_lo), 0.5 * (l_hi - l_lo)
    s = theta / delta
    rho = 1.0 / s
    r = b.copy() if x0 is None else b - Amul(x0)
    d = dinv * r / theta
    x = d.copy() if x0 is None else x0 + d
    for _ in range(2, degree + 1):
        r = b - Amul(x)
        rho_n = 1.0 / (2.0 * s - rho)
        d = rho_n * rho * d + (2.0 * rho_n / delta) * (dinv * r)
        x = x + d
        rho = rho_n
    return x


def vcycle(levels, transfers, b, degree, coarse_degree, lo=0.08, hi=1.2, level=0):
    """Symmetric V-cycle with zero initial guess.

    levels[l] = (A_l, dinv_l, lambda_l); transfers[l] = P_l (fine l <- coarse l+1),
    restriction = P_l^T.  Pre- and post-smoothing use `degree`; the coarsest
    level is a Chebyshev smoothing of `coarse_degree` from zero."""
    A, dinv, lam = levels[level]
    if level == len(levels) - 1:
        return chebyshev(A, dinv, b, None, lam, coarse_degree, lo, hi)
    x = chebyshev(A, dinv, b, None, lam, degree, lo, hi)
    r = b - A @ x
    P = transfers[level]
    xc = vcycle(levels, transfers, P.T @ r, degree, coarse_degree, lo, hi, level + 1)
    x = x + P @ xc
    return chebyshev(A, dinv, b, x, lam, degree, lo, hi)


def fast_diag_solve(M1s, K1s, alpha, sigma, b):
    """Solve (alpha Mz(x)My(x)Mx + sigma [Mz(x)My(x)Kx + Mz(x)Ky(x)Mx + Kz(x)My(x)Mx]) x = b
    (x the fastest index) by the generalised eigenpairs K1 V = M1 V Lambda,
    V^T M1 V = I, of each axis: x = V3 diag(1/(alpha + sigma(li+lj+lk))) V3^T b."""
    lams, Vs = [], []
    for M1, K1 in zip(M1s, K1s):
        lam, V = sla.eigh(K1, M1)
        lams.append(lam)
        Vs.append(V)
    Vx, Vy, Vz = Vs
    lx, ly, lz = lams
    nx, ny, nz = len(lx), len(ly), len(lz)
    B = b.reshape(nz, ny, nx)
    T = np.einsum("ia,jb,kc,kji->cba", Vx, Vy, Vz, B)
    T /= alpha + sigma * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :])
    X = np.einsum("ia,jb,kc,cba->kji", Vx, Vy, Vz, T)
    return X.reshape(-1)


def assemble_1d(p, n, L, kind="gll", q=None):
    """Global 1D mass and stiffness on n elements of length L/n (reference
    matrices scaled by h/2 and 2/h)."""
    from . import basis, quadrature
    nodes, _ = quadrature.gll(p)
    pts, w = quadrature.rule(kind, p, q)
    B = basis.lagrange(nodes, pts)
    D = basis.lagrange_deriv(nodes, pts)
    M1 = np.einsum("k,ka,kb->ab", w, B, B)
    K1 = np.einsum("k,ka,kb->ab", w, D, D)
    h = L / n
    N = p * n + 1
    M = np.zeros((N, N))
    K = np.zeros((N, N))
    for e in range(n):
        s = slice(p * e, p * e + p + 1)
        M[s, s] += 0.5 * h * M1
        K[s, s] += (2.0 / h) * K1
    return M, K
