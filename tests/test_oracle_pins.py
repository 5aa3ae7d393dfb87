"""Pins of the CPU oracle against things other than itself: closed forms,
library routines, invariants of the continuous problem, exact reproduction and
convergence rates, and the DOF counts the paper prints.  CPU only."""
import json
import math
import os

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import basis, mesh, multigrid, operator, quadrature, solvers, adjoint, ionic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _ev(s):
    return float(eval(s, {"sqrt": math.sqrt}))


# --- 1D rules -------------------------------------------------------------------

def test_quadrature_closed_forms():
    g = json.load(open(os.path.join(GOLD, "quadrature_closed_forms.json")))
    for p, d in g["gll"].items():
        x, w = quadrature.gll(int(p))
        np.testing.assert_allclose(x, [_ev(s) for s in d["x"]], atol=1e-15)
        np.testing.assert_allclose(w, [_ev(s) for s in d["w"]], rtol=1e-14)
    for q, d in g["gauss"].items():
        x, w = quadrature.gauss(int(q))
        np.testing.assert_allclose(x, [_ev(s) for s in d["x"]], atol=1e-15)
        np.testing.assert_allclose(w, [_ev(s) for s in d["w"]], rtol=1e-14)


@pytest.mark.parametrize("q", range(1, 14))
def test_gauss_matches_numpy(q):
    x, w = quadrature.gauss(q)
    xr, wr = npleg.leggauss(q)
    np.testing.assert_allclose(x, xr, atol=2e-15)
    np.testing.assert_allclose(w, wr, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("p", range(1, 12))
def test_gll_exactness_degree(p):
    """LGL with p+1 points is exact up to degree 2p-1 and not at 2p (Section 3)."""
    x, w = quadrature.gll(p)
    for m in range(2 * p):
        exact = 2.0 / (m + 1) if m % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** m) - exact) < 1e-14
    assert abs(np.sum(w * x ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-9
    # interior nodes are the roots of P_p' (numpy's Legendre series, independent)
    dP = npleg.legder(np.eye(p + 1)[p])
    np.testing.assert_allclose(npleg.legval(x[1:-1], dP), 0.0, atol=1e-12 * p * p)


@pytest.mark.parametrize("q", range(1, 12))
def test_gauss_exactness_degree(q):
    x, w = quadrature.gauss(q)
    for m in range(2 * q):
        exact = 2.0 / (m + 1) if m % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** m) - exact) < 1e-14
    assert abs(np.sum(w * x ** (2 * q)) - 2.0 / (2 * q + 1)) > 1e-8


# --- Lagrange basis -------------------------------------------------------------

@pytest.mark.parametrize("p", range(1, 10))
def test_lagrange_properties(p):
    nodes, _ = quadrature.gll(p)
    xs = np.linspace(-1, 1, 37)
    L = basis.lagrange(nodes, xs)
    D = basis.lagrange_deriv(nodes, xs)
    np.testing.assert_allclose(L.sum(1), 1.0, atol=1e-13)
    np.testing.assert_allclose(D.sum(1), 0.0, atol=1e-11 * p * p)
    np.testing.assert_array_equal(basis.lagrange(nodes, nodes), np.eye(p + 1))
    # interpolation and differentiation are exact on polynomials of degree p
    c = np.arange(1, p + 2) / 7.0
    f = npleg.legval(nodes, c)
    np.testing.assert_allclose(L @ f, npleg.legval(xs, c), atol=1e-12)
    np.testing.assert_allclose(D @ f, npleg.legval(xs, npleg.legder(c)), atol=1e-10 * p * p)


@pytest.mark.parametrize("p", range(1, 10))
def test_gll_derivative_closed_form(p):
    """D_ij = P_p(x_i)/(P_p(x_j)(x_i-x_j)), D_00 = -p(p+1)/4, D_pp = p(p+1)/4,
    0 otherwise (spectral-methods text cited in Section 3), with P_p from numpy."""
    x, _ = quadrature.gll(p)
    Pp = npleg.legval(x, np.eye(p + 1)[p])
    ref = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            if i != j:
                ref[i, j] = Pp[i] / (Pp[j] * (x[i] - x[j]))
    ref[0, 0] = -p * (p + 1) / 4.0
    ref[p, p] = p * (p + 1) / 4.0
    np.testing.assert_allclose(basis.lagrange_deriv(x, x), ref, atol=1e-12 * p * p)


def test_1d_matrices_p2():
    g = json.load(open(os.path.join(GOLD, "quadrature_closed_forms.json")))["matrices_p2"]
    nodes, wl = quadrature.gll(2)
    D = basis.lagrange_deriv(nodes, nodes)
    K = D.T @ np.diag(wl) @ D
    np.testing.assert_allclose(6 * K, g["gll_stiffness_times_6"], atol=1e-13)
    xg, wg = quadrature.gauss(3)
    B = basis.lagrange(nodes, xg)
    np.testing.assert_allclose(15 * B.T @ np.diag(wg) @ B, g["gauss3_mass_times_15"], atol=1e-13)
    np.testing.assert_allclose(3 * np.diag(wl), g["gll_mass_times_3"], atol=1e-14)


# --- element matrices -----------------------------------------------------------

def _ref_1d(p, kind, q=None):
    nodes, _ = quadrature.gll(p)
    pts, w = quadrature.rule(kind, p, q)
    B = basis.lagrange(nodes, pts)
    D = basis.lagrange_deriv(nodes, pts)
    return B.T @ np.diag(w) @ B, D.T @ np.diag(w) @ D


@pytest.mark.parametrize("p,kind,q", [(1, "gll", None), (2, "gll", None), (3, "gll", None),
                                      (2, "gauss", 3), (3, "gauss", 5), (4, "gll", None)])
def test_element_kronecker_closed_form(p, kind, q):
    """Affine cube of side h, sigma = I: M_e = (h/2)^3 M1(x)M1(x)M1 and
    K_e = (h/2) [M1(x)M1(x)K1 + M1(x)K1(x)M1 + K1(x)M1(x)M1] (x fastest)."""
    h = 0.7
    spec = synth.BoxSpec(p=p, n=(1, 1, 1), length=(h, h, h), quad=kind, nq1d=q or 0)
    prob = operator.Problem(spec)
    M, K = prob.elem_matrices(np.array([0]))
    M1, K1 = _ref_1d(p, kind, q)
    kr = np.kron
    np.testing.assert_allclose(M[0], (h / 2) ** 3 * kr(M1, kr(M1, M1)), atol=1e-15)
    Kref = (h / 2) * (kr(M1, kr(M1, K1)) + kr(M1, kr(K1, M1)) + kr(K1, kr(M1, M1)))
    np.testing.assert_allclose(K[0], Kref, atol=1e-13)


@pytest.mark.parametrize("p", range(1, 8))
def test_sem_mass_lumping_is_sem_ni_mass(p):
    """Row sums of the SEM (Gauss p+1) mass equal the SEM-NI diagonal mass on
    affine elements (Section 3: the lumped SEM mass is the SEM-NI mass)."""
    spec = synth.BoxSpec(p=p, n=(1, 1, 1), length=(1.3, 0.9, 1.1))
    Mg, _ = operator.Problem(spec, quad="gauss", q=p + 1).elem_matrices(np.array([0]))
    Ml, _ = operator.Problem(spec).elem_matrices(np.array([0]))
    np.testing.assert_allclose(Mg[0].sum(1), np.diag(Ml[0]), rtol=1e-13)
    np.testing.assert_allclose(Ml[0], np.diag(np.diag(Ml[0])), atol=1e-16)


def test_q1_equivalences():
    """Q1-SEM is Q1-FEM (exact mass (h/6)[[2,1],[1,2]] per axis); Q1-SEM-NI is
    Q1-FEM with the trapezoidal rule (mass (h/2) I per axis) (Section 3)."""
    h = 0.5
    spec = synth.BoxSpec(p=1, n=(1, 1, 1), length=(h, h, h))
    Mg, _ = operator.Problem(spec, quad="gauss", q=2).elem_matrices(np.array([0]))
    Ml, _ = operator.Problem(spec).elem_matrices(np.array([0]))
    m_fem = (h / 6) * np.array([[2, 1], [1, 2]])
    m_trap = (h / 2) * np.eye(2)
    kr = np.kron
    np.testing.assert_allclose(Mg[0], kr(m_fem, kr(m_fem, m_fem)), atol=1e-16)
    np.testing.assert_allclose(Ml[0], kr(m_trap, kr(m_trap, m_trap)), atol=1e-16)


# --- global operator invariants -------------------------------------------------

def _slab_small(p=3, quad="gll", q=0):
    return synth.slab(p, (5, 3, 2), quad=quad, nq1d=q)


@pytest.mark.parametrize("quad,q", [("gll", 0), ("gauss", 4), ("gauss", 5)])
def test_global_invariants_sheared_slab(quad, q):
    spec = _slab_small(3, quad, q)
    prob = operator.Problem(spec)
    A, M, K = prob.assemble()
    ones = np.ones(prob.n_dof)
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    assert np.max(np.abs(K @ ones)) < 1e-13 * abs(K).max()
    # the shear keeps the volume 20*7*3 = 420 exactly for every p (the
    # interpolated displacement vanishes at both ends of the slab)
    assert abs(ones @ (M @ ones) - 420.0) < 1e-10


def test_dirichlet_energy_of_linear_functions():
    """u = c.x is in the isoparametric space; for constant isotropic sigma,
    u^T K u = s |c|^2 |Omega| (here on the sheared slab)."""
    spec = _slab_small(3).with_(fiber=False, sigma=(0.3, 0.3, 0.3))
    prob = operator.Problem(spec)
    _, _, K = prob.assemble()
    c = np.array([0.3, -1.2, 0.7])
    u = prob.mesh.xyz @ c
    assert abs(u @ (K @ u) - 0.3 * (c @ c) * 420.0) < 1e-9 * 0.3 * (c @ c) * 420.0


@pytest.mark.parametrize("quad,q", [("gll", 0), ("gauss", 5)])
def test_anisotropic_energy_of_linear_functions(quad, q):
    """With a uniform fiber f (theta0 = theta1), sigma = sigma_t I + (sigma_l -
    sigma_t) f f^T is constant and u = c.x gives u^T K u = c^T sigma c |Omega|
    exactly (here on the sheared slab): pins the fiber term of the tensor."""
    th = 0.7
    sl, st = 0.17, 0.019
    spec = _slab_small(3, quad, q).with_(theta0=th, theta1=th, sigma=(sl, st, st))
    prob = operator.Problem(spec)
    _, _, K = prob.assemble()
    f = np.array([math.cos(th), math.sin(th), 0.0])
    sigma = st * np.eye(3) + (sl - st) * np.outer(f, f)
    for c in (np.array([0.3, -1.2, 0.7]), np.array([1.0, 0.0, 0.0])):
        u = prob.mesh.xyz @ c
        ref = (c @ sigma @ c) * 420.0
        assert abs(u @ (K @ u) - ref) < 1e-10 * ref


@pytest.mark.parametrize("quad,q", [("gll", 0), ("gauss", 4)])
def test_orthotropic_energy_along_principal_directions(quad, q):
    """With a uniform fiber a and sheet s (Section 2: the tensor has the
    eigenpairs (sigma_l, a), (sigma_t, s), (sigma_n, a x s)), u = c.x has
    u^T K u = |Omega| sum_i sigma_i (c . e_i)^2 over that frame: pins the sheet
    and cross-fiber terms (a swap of sigma_t and sigma_n, or a sheet left
    unnormalised, fails)."""
    th = 0.4
    sl, st, sn = 0.17, 0.05, 0.011
    spec = _slab_small(3, quad, q).with_(theta0=th, theta1=th, sheet=True, sigma=(sl, st, sn))
    prob = operator.Problem(spec)
    assert prob.mesh.sheet is not None
    _, _, K = prob.assemble()
    a = np.array([math.cos(th), math.sin(th), 0.0])
    s_ = np.array([-math.sin(th), math.cos(th), 0.0])
    n_ = np.array([0.0, 0.0, 1.0])
    for c, ref in ((a, sl), (s_, st), (n_, sn),
                   (0.3 * a - 1.2 * s_ + 0.7 * n_, 0.09 * sl + 1.44 * st + 0.49 * sn)):
        u = prob.mesh.xyz @ c
        assert abs(u @ (K @ u) - ref * 420.0) < 1e-10 * ref * 420.0


def test_paper_slab_workload_sizes():
    """The paper-shaped slab workload has the DOF counts the paper tabulates,
    and its orthotropic frame is (e_x, e_y, e_z)."""
    gold = json.load(open(os.path.join(GOLD, "paper_slab_dofs.json")))
    for p in (1, 2, 3, 4):
        spec = synth.paper_slab(p)
        assert spec.n_dof == gold["dofs"][str(p)]
    m = mesh.box(synth.paper_slab(1).with_(n=(4, 2, 2)))
    np.testing.assert_array_equal(m.fiber, np.tile([1.0, 0.0, 0.0], (m.n_dof, 1)))
    np.testing.assert_array_equal(m.sheet, np.tile([0.0, 1.0, 0.0], (m.n_dof, 1)))


def _rotation(a, b, c):
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Ry = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    Rx = np.array([[1, 0, 0], [0, math.cos(c), -math.sin(c)], [0, math.sin(c), math.cos(c)]])
    return Rz @ Ry @ Rx


@pytest.mark.parametrize("quad,q", [("gll", 0), ("gauss", 5)])
def test_rotation_invariance(quad, q):
    """Rotating coordinates and fibers together leaves K and M unchanged; a
    swapped J^{-1}/J^{-T} or a wrong fiber contraction breaks this."""
    spec = _slab_small(3, quad, q)
    prob = operator.Problem(spec)
    el = np.arange(spec.n_elem)
    M0, K0 = prob.elem_matrices(el)
    R = _rotation(0.4, -0.9, 1.3)
    prob.mesh.xyz = prob.mesh.xyz @ R.T
    prob.mesh.fiber = prob.mesh.fiber @ R.T
    M1, K1 = prob.elem_matrices(el)
    np.testing.assert_allclose(M1, M0, atol=1e-13 * abs(M0).max())
    np.testing.assert_allclose(K1, K0, atol=1e-12 * abs(K0).max())


def test_scaling():
    """Scaling coordinates by s scales M by s^3 and K by s."""
    spec = _slab_small(2)
    prob = operator.Problem(spec)
    el = np.arange(spec.n_elem)
    M0, K0 = prob.elem_matrices(el)
    prob.mesh.xyz = prob.mesh.xyz * 1.7
    M1, K1 = prob.elem_matrices(el)
    np.testing.assert_allclose(M1, 1.7 ** 3 * M0, rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(K1, 1.7 * K0, rtol=1e-12, atol=1e-14)


def test_r1_equals_r2_and_rows():
    spec = _slab_small(3)
    prob = operator.Problem(spec)
    A, _, _ = prob.assemble()
    x = synth.uniform(0, prob.n_dof)
    y1 = A @ x
    y2 = prob.apply_elementwise(x)
    np.testing.assert_allclose(y2, y1, atol=1e-13 * np.abs(y1).max())
    rows = np.array([0, 7, prob.n_dof // 2, prob.n_dof - 1, 123])
    y3 = operator.apply_rows(spec, lambda g: x[g], rows)
    np.testing.assert_allclose(y3, y1[rows], atol=1e-13 * np.abs(y1).max())
    np.testing.assert_allclose(prob.diagonal(), A.diagonal(), rtol=1e-13)


def test_spd_and_lanczos_bound():
    spec = _slab_small(2)
    prob = operator.Problem(spec)
    A, _, _ = prob.assemble()
    d = A.diagonal()
    Ad = (A.multiply(1 / np.sqrt(d)[:, None]).multiply(1 / np.sqrt(d)[None, :])).tocsr()
    ev = np.linalg.eigvalsh(Ad.toarray())
    assert ev.min() > 0
    lam = solvers.lanczos_lambda_max(A, 1 / d, synth.uniform(3, prob.n_dof), iters=10)
    assert lam <= ev.max() * (1 + 1e-12)
    assert lam >= 0.9 * ev.max()


# --- solves ---------------------------------------------------------------------

@pytest.mark.parametrize("p,kind,q,n,L", [
    (2, "gll", None, (4, 4, 4), (1.0, 1.0, 1.0)),            # the tiny unit-cube workload
    (3, "gll", None, (3, 2, 4), (1.3, 0.7, 2.1)),
    (2, "gauss", 3, (2, 3, 2), (1.0, 2.0, 0.5)),
    (3, "gauss", 5, (2, 2, 3), (0.8, 0.8, 1.5))])
def test_fast_diagonalisation_matches_assembled_solve(p, kind, q, n, L):
    spec = synth.BoxSpec(p=p, n=n, length=L, quad=kind, nq1d=q or 0, sigma=(0.6, 0.6, 0.6),
                         alpha=1.7)
    prob = operator.Problem(spec)
    A, _, _ = prob.assemble()
    b = synth.uniform(1, prob.n_dof)
    x = spla.spsolve(A.tocsc(), b)
    M1s, K1s = zip(*[solvers.assemble_1d(p, n[i], L[i], kind, q) for i in range(3)])
    xf = solvers.fast_diag_solve(M1s, K1s, 1.7, 0.6, b)
    np.testing.assert_allclose(x, xf, atol=1e-12 * np.abs(xf).max())


@pytest.mark.parametrize("p,kind", [(3, "gll"), (4, "gll"), (3, "gauss"), (4, "gauss")])
def test_exact_polynomial_reproduction(p, kind):
    """u = g(x)+g(y)+g(z), g(t) = 3t^2-2t^3 (zero normal derivative on the unit
    cube) is in Q_p for p >= 3 and every integral is exact, so the discrete
    solution of alpha u - s Lap u = f equals u at the nodes."""
    alpha, s = 1.7, 0.4
    spec = synth.BoxSpec(p=p, n=(2, 3, 2), quad=kind, alpha=alpha, sigma=(s, s, s))
    prob = operator.Problem(spec)
    A, M, _ = prob.assemble()
    g = lambda t: 3 * t ** 2 - 2 * t ** 3
    u_fn = lambda X: g(X[..., 0]) + g(X[..., 1]) + g(X[..., 2])
    f_fn = lambda X: alpha * u_fn(X) - s * ((6 - 12 * X[..., 0]) + (6 - 12 * X[..., 1]) + (6 - 12 * X[..., 2]))
    b = load_vector(prob, f_fn)
    x = spla.spsolve(A.tocsc(), b)
    np.testing.assert_allclose(x, u_fn(prob.mesh.xyz), atol=1e-12)


def load_vector(prob, f_fn):
    """b_i = sum_e sum_k W|J| f(X(xi_k)) phi_i(xi_k), by the oracle's quadrature."""
    nodes, _ = quadrature.gll(prob.p)
    Phi, _ = basis.basis3(nodes, prob.pts)
    map_nodes, _ = quadrature.gll(prob.map_p)
    Phi_m, _ = basis.basis3(map_nodes, prob.pts)
    b = np.zeros(prob.n_dof)
    for el in prob.chunks():
        geo = prob.elem_geometry(el)
        Xq = np.einsum("eir,ki->ekr", prob.mesh.xyz[prob.mesh.elem_dof[el]], Phi_m)
        be = np.einsum("ek,ki->ei", geo.WJ * f_fn(Xq), Phi)
        np.add.at(b, prob.elem_dof[el].reshape(-1), be.reshape(-1))
    return b


def _warp(xyz, eps):
    """Interior warping that keeps the unit cube's faces in place."""
    s = np.sin(np.pi * xyz[:, 0]) * np.sin(np.pi * xyz[:, 1]) * np.sin(np.pi * xyz[:, 2])
    return eps * np.stack([s, 0.7 * s, -0.5 * s], axis=1)


@pytest.mark.slow
@pytest.mark.parametrize("p", [2, 3])
def test_convergence_rate_curved(p):
    """Manufactured u = cos(pi x)cos(pi y)cos(pi z) on a warped unit-cube mesh:
    the nodal error decays like h^{p+1} (the SEM estimate of Section 3 gives
    h^p in H1; the nodal/L2 error is one order higher)."""
    alpha, s = 1.0, 1.0
    u_fn = lambda X: np.cos(np.pi * X[..., 0]) * np.cos(np.pi * X[..., 1]) * np.cos(np.pi * X[..., 2])
    f_fn = lambda X: (alpha + 3 * np.pi ** 2 * s) * u_fn(X)
    errs = []
    for n in (2, 4):
        spec = synth.BoxSpec(p=p, n=(n, n, n), alpha=alpha, sigma=(s, s, s))
        base = operator.Problem(spec)
        prob = operator.Problem(spec, jitter=_warp(base.mesh.xyz, 0.04))
        A, M, _ = prob.assemble()
        x = spla.spsolve(A.tocsc(), load_vector(prob, f_fn))
        e = x - u_fn(prob.mesh.xyz)
        errs.append(math.sqrt(e @ (M @ e)))
    rate = math.log2(errs[0] / errs[1])
    assert rate > p + 1 - 0.6, (errs, rate)


def test_p_convergence_is_faster_than_algebraic():
    """Error at fixed h drops by large factors as p grows (Section 3)."""
    alpha, s = 1.0, 1.0
    u_fn = lambda X: np.cos(np.pi * X[..., 0]) * np.cos(np.pi * X[..., 1]) * np.cos(np.pi * X[..., 2])
    f_fn = lambda X: (alpha + 3 * np.pi ** 2 * s) * u_fn(X)
    errs = []
    for p in (2, 3, 4, 5):
        spec = synth.BoxSpec(p=p, n=(2, 2, 2), alpha=alpha, sigma=(s, s, s))
        prob = operator.Problem(spec)
        A, M, _ = prob.assemble()
        x = spla.spsolve(A.tocsc(), load_vector(prob, f_fn))
        e = x - u_fn(prob.mesh.xyz)
        errs.append(math.sqrt(e @ (M @ e)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(r > 4 for r in ratios), (errs, ratios)


def test_paper_slab_dof_counts():
    g = json.load(open(os.path.join(GOLD, "paper_slab_dofs.json")))
    for p, n in g["dofs"].items():
        spec = synth.BoxSpec(p=int(p), n=tuple(g["cells"]))
        assert spec.n_dof == n
        assert mesh.elem_dof_map(int(p), tuple(g["cells"])).max() + 1 == n if int(p) <= 2 else True


def test_cg_matches_direct():
    spec = _slab_small(3)
    prob = operator.Problem(spec)
    A, _, _ = prob.assemble()
    b = synth.uniform(2, prob.n_dof)
    xd = spla.spsolve(A.tocsc(), b)
    x, it, rn = solvers.cg(A, b, rtol=1e-13)
    np.testing.assert_allclose(x, xd, atol=1e-10 * np.abs(xd).max())


# --- multigrid pieces -----------------------------------------------------------

@pytest.mark.parametrize("pf,pc", [(4, 2), (2, 1), (7, 3), (3, 1)])
def test_p_prolongation_reproduces_polynomials(pf, pc):
    n = (2, 3, 2)
    P = multigrid.prolongation_p(n, pf, pc)
    Xf = mesh.box(synth.BoxSpec(p=pf, n=n)).xyz
    Xc = mesh.box(synth.BoxSpec(p=pc, n=n)).xyz
    f = lambda X: (X[:, 0] ** pc) * (1 + X[:, 1]) ** pc - 2 * X[:, 2] ** pc + X[:, 0] * X[:, 1] * X[:, 2]
    np.testing.assert_allclose(P @ f(Xc), f(Xf), atol=1e-12)
    assert abs(P.sum(1).A1 - 1).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 4])
def test_h_prolongation_reproduces_polynomials(p):
    nf = (4, 2, 6)
    P = multigrid.prolongation_h(nf, p)
    Xf = mesh.box(synth.BoxSpec(p=p, n=nf)).xyz
    Xc = mesh.box(synth.BoxSpec(p=p, n=(2, 1, 3))).xyz
    f = lambda X: (X[:, 0] ** p) * (1 + X[:, 1]) ** p - 2 * X[:, 2] ** p + X[:, 0] * X[:, 2]
    if p == 1:
        f = lambda X: 1 + X[:, 0] - 2 * X[:, 1] + 3 * X[:, 2]
    np.testing.assert_allclose(P @ f(Xc), f(Xf), atol=1e-12)


def test_galerkin_identity_p_levels():
    """Affine mesh, exact (Gauss) quadrature: A_c = P^T A_f P."""
    spec = synth.BoxSpec(p=4, n=(2, 2, 1), length=(1.0, 0.6, 0.9), quad="gauss", nq1d=5,
                         sigma=(0.5, 0.5, 0.5), alpha=2.0)
    Af, _, _ = operator.Problem(spec).assemble()
    Ac, _, _ = operator.Problem(spec, dof_p=2, quad="gauss", q=3).assemble()
    P = multigrid.prolongation_p(spec.n, 4, 2)
    np.testing.assert_allclose((P.T @ Af @ P).toarray(), Ac.toarray(), atol=1e-12)


def _chebyshev_T(k, x):
    return np.cosh(k * np.arccosh(x)) if x >= 1 else np.cos(k * np.arccos(x))


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_chebyshev_error_polynomial(k):
    """From x0 = 0 with D = I, the error in each eigencomponent is multiplied by
    T_k((theta - lam)/delta) / T_k(theta/delta) (closed form)."""
    lam = np.linspace(0.05, 2.0, 40)
    A = np.diag(lam)
    xs = synth.uniform(5, 40)
    b = A @ xs
    lmax = 2.0
    x = solvers.chebyshev(A, np.ones(40), b, None, lmax, k)
    lo, hi = 0.08 * lmax * 1.0, 1.2 * lmax
    th, de = (hi + lo) / 2, (hi - lo) / 2
    fac = np.array([_chebyshev_T(k, (th - l) / de) for l in lam]) / _chebyshev_T(k, th / de)
    np.testing.assert_allclose(xs - x, fac * xs, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_chebyshev_equals_damped_jacobi_over_its_roots(k):
    """The degree-k Chebyshev smoother is also the product of k damped-Jacobi
    steps with weights 1/r over the roots r of its polynomial (the factored form
    the GPU smoother runs): after k steps both reach the same iterate, from zero
    and from a nonzero start, with a non-identity diagonal; taken from the
    largest root down, no partial product exceeds 1 in magnitude on [0, hi]."""
    rng = np.random.default_rng(k)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    A = Q @ np.diag(np.linspace(0.1, 3.0, 30)) @ Q.T
    A = A + np.diag(np.linspace(1.0, 2.0, 30))
    dinv = 1.0 / np.diag(A)
    Dh = np.diag(np.sqrt(dinv))
    lmax = np.linalg.eigvalsh(Dh @ A @ Dh).max()
    lo, hi = 0.08 * lmax, 1.2 * lmax
    th, de = (hi + lo) / 2, (hi - lo) / 2
    roots = [th + de * np.cos((2 * j + 1) * np.pi / (2 * k)) for j in range(k)]
    assert all(roots[j] > roots[j + 1] for j in range(k - 1))
    b = synth.uniform(11, 30)
    for x0 in (None, synth.uniform(12, 30)):
        ref = solvers.chebyshev(A, dinv, b, x0, lmax, k)
        x = np.zeros(30) if x0 is None else x0.copy()
        for r in roots:
            x = x + (1.0 / r) * dinv * (b - A @ x)
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    lam = np.linspace(0.0, hi, 501)
    prod = np.ones_like(lam)
    for r in roots:
        prod = prod * (1 - lam / r)
        assert np.abs(prod).max() <= 1.0 + 1e-12


def test_vcycle_is_symmetric_positive():
    spec = synth.slab(4, (4, 2, 2))
    levels, transfers = [], []
    for pl in (4, 2, 1):
        prob = operator.Problem(spec, dof_p=pl)
        A, _, _ = prob.assemble()
        dinv = 1 / A.diagonal()
        lam = solvers.lanczos_lambda_max(A, dinv, synth.uniform(9, prob.n_dof))
        levels.append((A, dinv, lam))
    transfers = [multigrid.prolongation_p(spec.n, 4, 2), multigrid.prolongation_p(spec.n, 2, 1)]
    N = levels[0][0].shape[0]
    V = lambda r: solvers.vcycle(levels, transfers, r, 3, 6)
    b1, b2 = synth.uniform(10, N), synth.uniform(11, N)
    assert abs(V(b1) @ b2 - b1 @ V(b2)) < 1e-12 * abs(V(b1) @ b2)
    assert V(b1) @ b1 > 0
    # as a preconditioner it converges fast and to the direct solution
    A = levels[0][0]
    x, it, _ = solvers.cg(A, b1, rtol=1e-12, M=V)
    np.testing.assert_allclose(x, spla.spsolve(A.tocsc(), b1), atol=1e-9 * abs(x).max())
    assert it < 25


def _smoother_matrix(A, dinv, lam, k):
    """The pre-smoother from zero as an explicit matrix S (x = S b), column by
    column from the oracle's Chebyshev routine (pinned above by its closed-form
    error polynomial)."""
    n = A.shape[0]
    return np.stack([solvers.chebyshev(A, dinv, e, None, lam, k) for e in np.eye(n)], axis=1)


def _exact_cycle_hierarchy(A0, b, x_star, k, rng, m1=6):
    """Levels and transfers on which a correct V-cycle returns the exact
    solution x* of A0 x = b (b = A0 x*), by construction:
      * level 0 -> 1: the first column of P0 is the error left by pre-smoothing,
        (I - S0 A0) x*; the rest are random.  A1 = P0^T A0 P0 (Galerkin).
      * level 1 -> 2: the restricted residual is g = P0^T (b - A0 S0 b), whose
        exact coarse solution y* = A1^{-1} g is in the coarse space; P1 is the
        single column (I - S1 A1) y*, the error pre-smoothing leaves on level 1.
      * level 2 is 1x1 with lambda = 1/0.64: Chebyshev of degree 1 from zero is
        then D^{-1} b / theta with theta = 1, i.e. the exact solve.
    Pre-smoothing leaves an error in the range of the prolongation, the exact
    coarse correction removes it, and post-smoothing keeps the exact solution."""
    n0 = A0.shape[0]
    d0 = 1.0 / np.diag(A0)
    lam0 = np.linalg.eigvals(d0[:, None] * A0).real.max()
    S0 = _smoother_matrix(A0, d0, lam0, k)
    P0 = np.column_stack([x_star - S0 @ (A0 @ x_star), rng.standard_normal((n0, m1 - 1))])
    A1 = P0.T @ A0 @ P0
    d1 = 1.0 / np.diag(A1)
    lam1 = np.linalg.eigvals(d1[:, None] * A1).real.max()
    S1 = _smoother_matrix(A1, d1, lam1, k)
    g = P0.T @ (b - A0 @ (S0 @ b))
    y_star = np.linalg.solve(A1, g)
    P1 = (y_star - S1 @ (A1 @ y_star))[:, None]
    A2 = P1.T @ A1 @ P1
    levels = [(A0, d0, lam0), (A1, d1, lam1), (A2, 1.0 / np.diag(A2), 1.0 / 0.64)]
    return levels, [P0, P1]


@pytest.mark.parametrize("k", [1, 3])
def test_vcycle_coarse_correction_is_exact_on_a_constructed_hierarchy(k):
    """Section 4.3's V-cycle: smooth, restrict the residual, correct with the
    prolongated coarse solution, smooth again.  On the hierarchy built by
    _exact_cycle_hierarchy every step is exact, so one cycle from zero returns
    x*; dropping, mis-scaling or mis-signing the coarse correction, restricting
    b instead of the residual, or skipping a level would leave an error of the
    size of x*.  Two-level and three-level cycles on an SPD matrix from the
    assembled operator."""
    spec = synth.slab(2, (2, 2, 1))
    A0 = operator.Problem(spec).assemble()[0].toarray()
    rng = np.random.default_rng(17 + k)
    x_star = rng.standard_normal(A0.shape[0])
    b = A0 @ x_star
    levels, transfers = _exact_cycle_hierarchy(A0, b, x_star, k, rng)
    x = solvers.vcycle(levels, transfers, b, k, 1)
    np.testing.assert_allclose(x, x_star, rtol=0, atol=1e-9 * np.abs(x_star).max())
    # two levels: level 1 solved exactly by making it the 1x1 coarsest level of a
    # hierarchy whose single coarse vector is the error pre-smoothing leaves
    d0, lam0 = levels[0][1], levels[0][2]
    S0 = _smoother_matrix(A0, d0, lam0, k)
    P = (x_star - S0 @ (A0 @ x_star))[:, None]
    Ac = P.T @ A0 @ P
    two = [levels[0], (Ac, 1.0 / np.diag(Ac), 1.0 / 0.64)]
    x2 = solvers.vcycle(two, [P], b, k, 1)
    np.testing.assert_allclose(x2, x_star, rtol=0, atol=1e-9 * np.abs(x_star).max())


def test_vcycle_beats_the_smoother_alone():
    """With a small mass coefficient the Jacobi-Chebyshev smoother alone leaves
    the smooth error: as a CG preconditioner it needs several times the
    iterations of the V-cycle on the p 4 -> 2 -> 1 hierarchy (Section 5 reports
    1.4-2.1 GMG iterations per solve, independent of h and p)."""
    spec = synth.slab(4, (8, 3, 2)).with_(alpha=0.01)
    levels = []
    for pl in (4, 2, 1):
        A = operator.Problem(spec, dof_p=pl).assemble()[0]
        dinv = 1 / A.diagonal()
        levels.append((A, dinv, solvers.lanczos_lambda_max(A, dinv, synth.uniform(9, A.shape[0]))))
    transfers = [multigrid.prolongation_p(spec.n, 4, 2), multigrid.prolongation_p(spec.n, 2, 1)]
    A, dinv, lam = levels[0]
    b = synth.uniform(3, A.shape[0])
    _, it_mg, _ = solvers.cg(A, b, rtol=1e-10, M=lambda r: solvers.vcycle(levels, transfers, r, 3, 6))
    sym = lambda r: solvers.chebyshev(A, dinv, b=r, x0=solvers.chebyshev(A, dinv, r, None, lam, 3),
                                      lam_max=lam, degree=3)
    _, it_sm, _ = solvers.cg(A, b, rtol=1e-10, M=sym)
    assert it_mg <= 20 and it_sm >= 3 * it_mg, (it_mg, it_sm)


# --- adjoint --------------------------------------------------------------------

def test_linearity_in_sigma_and_adjoint_fd():
    spec = synth.slab(2, (3, 2, 2))
    sig = synth.element_sigma(4, 1, spec.n_elem)[0]
    sig[:, 2] = sig[:, 1] * 1.3  # distinct sigma_n exercises the no-sheet reading
    prob = operator.Problem(spec, sigma=sig)
    f = synth.uniform(5, prob.n_dof)
    ut = synth.uniform(6, prob.n_dof) * 0.01
    L, g, lam, u = adjoint.loss_and_grad(prob, f, ut)
    h = 1e-6
    for e, c in [(0, 0), (5, 1), (11, 0), (7, 1)]:
        sp_, sm_ = sig.copy(), sig.copy()
        sp_[e, c] += h
        sm_[e, c] -= h
        Lp = adjoint.loss(operator.Problem(spec, sigma=sp_), f, ut)
        Lm = adjoint.loss(operator.Problem(spec, sigma=sm_), f, ut)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[e, c]) <= 1e-6 * max(abs(fd), 1e-3 * abs(g).max()), (e, c, fd, g[e, c])
    # without a sheet sigma_n does not enter
    assert np.all(g[:, 2] == 0)
    # A is exactly linear in sigma: A(2 sigma) - A(sigma) = K(sigma)
    A1, _, K1 = prob.assemble()
    A2, _, _ = operator.Problem(spec, sigma=2 * sig).assemble()
    assert abs((A2 - A1) - K1).max() < 1e-12 * abs(K1).max()


# --- ionic ----------------------------------------------------------------------

def test_aliev_panfilov_rest_and_rates():
    prm = synth.AP_PARAMS
    F, G = ionic.ap_rates(np.array([0.0]), np.array([0.0]), **prm)
    assert F[0] == 0.0 and G[0] == 0.0
    # hand evaluation at u = 0.5, w = 0.1
    u, w = 0.5, 0.1
    k, a = prm["k"], prm["a"]
    Fh = k * 0.5 * 0.5 * 0.35 - 0.05
    eps = prm["eps0"] + prm["mu1"] * 0.1 / 0.8
    Gh = eps * (-0.1 - k * 0.5 * (0.5 - 0.15 - 1))
    F, G = ionic.ap_rates(np.array([u]), np.array([w]), **prm)
    assert abs(F[0] - Fh) < 1e-15 and abs(G[0] - Gh) < 1e-15
    V = np.array([prm["v_rest"]])
    b, wn = ionic.imex_rhs_and_gate(V, np.zeros(1), np.zeros(1), np.array([2.0]), 0.05,
                                    synth.CHI, synth.CM, prm)
    assert abs(b[0] - 2.0 * (synth.CHI * synth.CM / 0.05) * prm["v_rest"]) < 1e-12
    assert wn[0] == 0.0


# --- BDF2 partitioned scheme (Section 3) ----------------------------------------

def _cell_rates(V, w, prm):
    """Single-cell AP model in mV and ms: dV/dt, dw/dt (no diffusion, no stimulus)."""
    u = (V - prm["v_rest"]) / prm["v_amp"]
    F, G = ionic.ap_rates(np.atleast_1d(u), np.atleast_1d(w), **prm)
    return (prm["v_amp"] / prm["t_scale"]) * F[0], G[0] / prm["t_scale"]


def _cell_run(scheme, dt, T, V0, w0, Vm1, wm1, prm):
    """March one cell (M = 1, K = 0) with the oracle's step functions."""
    chi, cm = synth.CHI, synth.CM
    one, zero = np.ones(1), np.zeros(1)
    V, w, Vo, wo = np.array([V0]), np.array([w0]), np.array([Vm1]), np.array([wm1])
    for _ in range(int(round(T / dt))):
        if scheme == "bdf2":
            b, wn = ionic.bdf2_rhs_and_gate(V, Vo, w, wo, zero, one, dt, chi, cm, prm)
            Vn = b / (1.5 * chi * cm / dt)
        else:
            b, wn = ionic.imex_rhs_and_gate(V, w, zero, one, dt, chi, cm, prm)
            Vn = b / (chi * cm / dt)
        Vo, wo, V, w = V, w, Vn, wn
    return V[0], w[0]


def test_bdf2_cell_converges_at_second_order():
    """The partitioned BDF2 step with the extrapolated potential is second-order
    accurate (Section 3); the first-order IMEX step first-order.  Reference: an
    adaptive Runge-Kutta solve of the same cell ODE at tight tolerance."""
    from scipy.integrate import solve_ivp
    prm = synth.AP_PARAMS
    y0 = (-30.0, 0.4)
    T = 1.0
    rhs = lambda t, y: list(_cell_rates(y[0], y[1], prm))
    ref = solve_ivp(rhs, (0.0, T), y0, method="DOP853", rtol=1e-13, atol=1e-13,
                    dense_output=True)
    VT = ref.sol(T)[0]
    err = {}
    for scheme in ("bdf2", "imex1"):
        err[scheme] = []
        for dt in (0.02, 0.01, 0.005):
            # exact history value at t = -dt for the two-step scheme
            back = solve_ivp(rhs, (0.0, -dt), y0, method="DOP853", rtol=1e-13, atol=1e-13)
            Vm1, wm1 = back.y[0, -1], back.y[1, -1]
            VTn, _ = _cell_run(scheme, dt, T, y0[0], y0[1], Vm1, wm1, prm)
            err[scheme].append(abs(VTn - VT))
    r2 = [np.log2(err["bdf2"][i] / err["bdf2"][i + 1]) for i in range(2)]
    r1 = [np.log2(err["imex1"][i] / err["imex1"][i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.3 for r in r2), (err, r2)
    assert all(0.8 < r < 1.3 for r in r1), (err, r1)


def test_bdf2_gate_linear_case_and_rest_state():
    """With mu1 = 0 the gating equation is linear: w = (4 w^n - w^{n-1} - h eps0 c) /
    (3 + h eps0); the rest state is a fixed point of the whole step."""
    prm = dict(synth.AP_PARAMS, mu1=0.0)
    rng = np.random.default_rng(3)
    u = rng.uniform(-0.1, 1.1, 50)
    wn, wm = rng.uniform(0, 2, 50), rng.uniform(0, 2, 50)
    dt = 0.05
    h = 2 * dt / prm["t_scale"]
    c = prm["k"] * u * (u - prm["a"] - 1.0)
    w_closed = (4 * wn - wm - h * prm["eps0"] * c) / (3 + h * prm["eps0"])
    w = ionic.bdf2_gate(u, wn, wm, dt, **prm)
    assert np.max(np.abs(w - w_closed)) < 1e-14
    prm = synth.AP_PARAMS
    V = np.full(3, prm["v_rest"])
    b, wnext = ionic.bdf2_rhs_and_gate(V, V, np.zeros(3), np.zeros(3), np.zeros(3),
                                       np.full(3, 2.0), dt, synth.CHI, synth.CM, prm)
    assert np.all(wnext == 0.0)
    # (3/2 alpha1 M + K) V = b is solved by V = v_rest (K annihilates constants)
    assert np.allclose(b, 2.0 * 1.5 * synth.CHI * synth.CM / dt * prm["v_rest"], rtol=1e-15)


def _tanh_series(n_steps, m, dt, width, amp, base=0.0, half=True):
    """V_n = base + amp tanh(s_n), s_n = (n - m - 1/2) dt / width (half=True: the
    steepest point sits at the midpoint of step m) or (n - m) dt / width (half=False:
    on the sample t_m, so steps m-1 and m are equally steep).  Built from |s| so
    that V is exactly antisymmetric about its centre whatever tanh's rounding."""
    k = np.arange(n_steps + 1) - m - (0.5 if half else 0.0)
    mag = amp * np.tanh(np.abs(k) * dt / width)
    return base + np.where(k < 0, -mag, mag)


def test_activation_time_is_steepest_point_of_tanh_upstrokes():
    """Section 5.1: tau = argmax_t |du/dt|.  For V = base + amp tanh((t - t0)/w)
    sampled every dt with t0 half-way between two samples, the steepest step is
    the one centred on the inflection point t0, so tau = t0 exactly; this holds
    for downstrokes (amp < 0) as for upstrokes, and on a DOF with a gentle
    upstroke followed by a steeper downstroke the downstroke wins."""
    dt, n_steps = 0.05, 200
    t = np.arange(n_steps + 1) * dt
    cols, tau_exact = [], []
    for m, w, amp, base in [(40, 0.2, 50.0, -35.0), (123, 0.9, 50.0, -35.0),
                            (7, 0.05, -60.0, 0.0), (170, 3.0, 1.0, -80.0)]:
        cols.append(_tanh_series(n_steps, m, dt, w, amp, base))
        tau_exact.append((m + 0.5) * dt)
    up = _tanh_series(n_steps, 30, dt, 1.0, 20.0)       # gentle upstroke at step 30
    down = _tanh_series(n_steps, 150, dt, 0.1, -45.0)   # steep downstroke at step 150
    cols.append(up + down)
    tau_exact.append(150.5 * dt)
    V = np.stack(cols, axis=1)
    tau, rate = ionic.activation_times(V, t)
    np.testing.assert_allclose(tau, tau_exact, rtol=0, atol=1e-12)
    # the largest rate is the difference quotient over the centred step
    assert abs(rate[0] - 2 * 50.0 * np.tanh(0.5 * dt / 0.2) / dt) < 1e-9
    # the crossing of a level below the inflection point comes earlier
    cross = np.full(V.shape[1], -1.0)
    for n in range(n_steps):
        cross = ionic.threshold_crossing_update(cross, V[n], V[n + 1], t[n], t[n + 1], -40.0)
    t_cross = tau_exact[0] - 0.2 * np.arctanh(0.1)
    assert abs(cross[0] - t_cross) < 0.5 * dt and cross[0] < tau[0] - 0.01


def test_activation_time_ties_take_the_first_step():
    """With the inflection point on a sample, the two steps around it have
    exactly equal |dV| (V is antisymmetric about it), and the earlier one is
    the activation step; a constant potential has no activation time.  The
    step is a power of two, so the time grid is exact and so are the ties."""
    dt, n_steps, m = 0.125, 60, 25
    t = np.arange(n_steps + 1) * dt
    V = np.stack([_tanh_series(n_steps, m, dt, 0.3, 40.0, half=False),
                  np.full(n_steps + 1, -80.0)], axis=1)
    q = np.abs(np.diff(V[:, 0])) / np.diff(t)
    assert q[m - 1] == q[m] == q.max()
    tau, rate = ionic.activation_times(V, t)
    assert abs(tau[0] - (m - 0.5) * dt) < 1e-12
    assert tau[1] == -1.0 and rate[1] == 0.0


def test_activation_running_form_equals_series_form_and_brute_force():
    """The one-step running maximum equals the whole-series definition, and
    both equal numpy's argmax (first occurrence) of |diff V| over random series
    with repeated values (ties) and a non-uniform time grid."""
    rng = np.random.default_rng(5)
    n_steps, n = 40, 300
    t = np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, n_steps)]) * 0.01
    V = np.round(rng.normal(size=(n_steps + 1, n)) * 3) * 2.0  # small integers: many ties
    tau, rate = ionic.activation_times(V, t)
    act, r = np.full(n, -1.0), np.zeros(n)
    for k in range(n_steps):
        act, r = ionic.activation_update(act, r, V[k], V[k + 1], t[k + 1], t[k + 1] - t[k])
    assert np.array_equal(act, tau) and np.array_equal(r, rate)
    q = np.abs(np.diff(V, axis=0)) / np.diff(t)[:, None]
    k = np.argmax(q, axis=0)
    mid = t[1:] - 0.5 * np.diff(t)
    moved = q.max(axis=0) > 0
    np.testing.assert_allclose(tau[moved], mid[k[moved]], rtol=0, atol=1e-15)
    assert np.all(tau[~moved] == -1.0)


def test_activation_time_converges_to_the_inflection_point():
    """For a smooth upstroke whose steepest point t* falls between samples, the
    discrete activation time is within dt/2 of t* and approaches it as dt -> 0."""
    ts = 1.2345
    f = lambda t: -80.0 + 50.0 * (1.0 + np.tanh((t - ts) / 0.07))
    errs = []
    for dt in (0.04, 0.02, 0.01, 0.005):
        t = np.arange(0.0, 3.0 + dt / 2, dt)
        tau, _ = ionic.activation_times(f(t)[:, None], t)
        errs.append(abs(tau[0] - ts))
        assert errs[-1] <= 0.5 * dt + 1e-12
    assert errs[-1] < errs[0]
