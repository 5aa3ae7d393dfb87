"""Planted mistakes in the oracle (on the CPU): each plausible error below must
make at least one of the pins in test_oracle_pins.py fail, so the pins are
strong enough to trust the oracle.  The mistakes are applied with monkeypatch
and never touch the GPU path."""
import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import adjoint, basis, multigrid, operator, quadrature, solvers


def _fails(fn):
    try:
        fn()
    except Exception:  # an assertion, or an error the mistake provokes
        return True
    return False


def _geometry_with(fix):
    orig = operator.geometry

    def wrapped(*a, **k):
        g = orig(*a, **k)
        return fix(g)
    return wrapped


MUTATIONS = {
    # derivative matrix transposed (D[k][a] read as D[a][k])
    "derivative transposed": (
        lambda mp: mp.setattr(basis, "lagrange_deriv",
                              (lambda orig: lambda n, x: orig(n, x).T if len(n) == len(x)
                               else orig(n, x))(basis.lagrange_deriv)),
        [lambda: pins.test_gll_derivative_closed_form(3),
         lambda: pins.test_exact_polynomial_reproduction(3, "gll")]),
    # J^{-1} where J^{-T} belongs (transposed inverse Jacobian)
    "inverse Jacobian transposed": (
        lambda mp: mp.setattr(operator, "geometry", _geometry_with(
            lambda g: operator.Geometry(WJ=g.WJ, Jinv=np.swapaxes(g.Jinv, -1, -2), f=g.f, s=g.s))),
        [lambda: pins.test_rotation_invariance("gll", 0),
         lambda: pins.test_dirichlet_energy_of_linear_functions()]),
    # sigma_l and sigma_t exchanged in the diffusion tensor
    "sigma_l and sigma_t swapped": (
        lambda mp: mp.setattr(operator, "sigma_tensor",
                              (lambda orig: lambda sig, f=None, s=None:
                               orig(sig[..., [1, 0, 2]], f, s))(operator.sigma_tensor)),
        [lambda: pins.test_anisotropic_energy_of_linear_functions("gll", 0)]),
    # sigma_t and sigma_n exchanged (sheet and cross-fiber directions mixed up)
    "sigma_t and sigma_n swapped": (
        lambda mp: mp.setattr(operator, "sigma_tensor",
                              (lambda orig: lambda sig, f=None, s=None:
                               orig(sig[..., [0, 2, 1]], f, s))(operator.sigma_tensor)),
        [lambda: pins.test_orthotropic_energy_along_principal_directions("gll", 0)]),
    # sheet not used (transversely isotropic tensor although a sheet is given)
    "sheet dropped": (
        lambda mp: mp.setattr(operator, "sigma_tensor",
                              (lambda orig: lambda sig, f=None, s=None: orig(sig, f, None))(
                                  operator.sigma_tensor)),
        [lambda: pins.test_orthotropic_energy_along_principal_directions("gauss", 4)]),
    # fiber direction not used (isotropic sigma_t I regardless of the fiber)
    "fiber term dropped": (
        lambda mp: mp.setattr(operator, "sigma_tensor",
                              (lambda orig: lambda sig, f=None, s=None: orig(sig, None, None))(
                                  operator.sigma_tensor)),
        [lambda: pins.test_anisotropic_energy_of_linear_functions("gauss", 5)]),
    # quadrature weight W|J| off by a factor (e.g. a reference-cube volume slip)
    "mass weight scaled": (
        lambda mp: mp.setattr(operator, "geometry", _geometry_with(
            lambda g: operator.Geometry(WJ=g.WJ * 1.01, Jinv=g.Jinv, f=g.f, s=g.s))),
        [lambda: pins.test_global_invariants_sheared_slab("gll", 0)]),
    # GLL weights from the wrong formula (one node's weight perturbed)
    "GLL weights wrong": (
        lambda mp: mp.setattr(quadrature, "gll",
                              (lambda orig: lambda p: (orig(p)[0], orig(p)[1] * np.r_[1.0, [1.0] * (p - 1), 1.001]))(
                                  quadrature.gll)),
        [lambda: pins.test_quadrature_closed_forms(),
         lambda: pins.test_gll_exactness_degree(3)]),
    # Chebyshev interval taken from [lo, hi] as fractions of 1 instead of lambda_max
    "Chebyshev interval": (
        lambda mp: mp.setattr(solvers, "chebyshev",
                              (lambda orig: lambda A, dinv, b, x0, lam, deg, lo=0.08, hi=1.2:
                               orig(A, dinv, b, x0, 1.0, deg, lo, hi))(solvers.chebyshev)),
        [lambda: pins.test_chebyshev_error_polynomial(3)]),
    # h-prolongation with the children's halves exchanged
    "h-prolongation halves swapped": (
        lambda mp: mp.setattr(multigrid, "prolongation_h",
                              (lambda orig: lambda n, p: orig(n, p)[::-1])(multigrid.prolongation_h)),
        [lambda: pins.test_h_prolongation_reproduces_polynomials(2)]),
    # adjoint gradient with the wrong sign
    "adjoint sign": (
        lambda mp: mp.setattr(adjoint, "grad_sigma",
                              (lambda orig: lambda prob, u, w: -orig(prob, u, w))(adjoint.grad_sigma)),
        [lambda: pins.test_linearity_in_sigma_and_adjoint_fd()]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    plant, checks = MUTATIONS[name]
    plant(monkeypatch)
    assert any(_fails(c) for c in checks), f"no pin caught: {name}"


def test_pins_pass_without_mistakes():
    """The same checks pass on the unmodified oracle (so a failure above is the mistake's)."""
    for _, checks in MUTATIONS.values():
        for c in checks:
            c()
