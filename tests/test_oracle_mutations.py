"""Planted mistakes in the oracle (on the CPU): each plausible error below must
make at least one of the pins in test_oracle_pins.py fail, so the pins are
strong enough to trust the oracle.  The mistakes are applied with monkeypatch
and never touch the GPU path."""
import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import adjoint, basis, ionic, multigrid, operator, quadrature, solvers


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


def _vcycle_with(correct=lambda x, Pxc: x + Pxc, restrict_residual=True):
    """The oracle's V-cycle with its coarse-grid step replaced (for planting
    mistakes): x <- correct(x, P xc), and b restricted in place of b - A x
    when restrict_residual is False."""
    def vc(levels, transfers, b, degree, coarse_degree, lo=0.08, hi=1.2, level=0):
        A, dinv, lam = levels[level]
        if level == len(levels) - 1:
            return solvers.chebyshev(A, dinv, b, None, lam, coarse_degree, lo, hi)
        x = solvers.chebyshev(A, dinv, b, None, lam, degree, lo, hi)
        r = b - A @ x if restrict_residual else b
        P = transfers[level]
        xc = vc(levels, transfers, P.T @ r, degree, coarse_degree, lo, hi, level + 1)
        x = correct(x, P @ xc)
        return solvers.chebyshev(A, dinv, b, x, lam, degree, lo, hi)
    return vc


def _activation_with(stamp="mid", absolute=True, ties="first"):
    """The oracle's activation time with one detail changed: the time stamp of
    the steepest step (its midpoint or its end), the absolute value of the
    derivative, or which step wins a tie."""
    def act(V_series, t_series):
        V, t = np.asarray(V_series), np.asarray(t_series)
        q = np.diff(V, axis=0) / np.diff(t)[:, None]
        q = np.abs(q) if absolute else q
        k = (np.argmax(q, axis=0) if ties == "first"
             else q.shape[0] - 1 - np.argmax(q[::-1], axis=0))
        when = 0.5 * (t[:-1] + t[1:]) if stamp == "mid" else t[1:]
        moved = q.max(axis=0) > 0
        return np.where(moved, when[k], -1.0), np.where(moved, q.max(axis=0), 0.0)
    return act


def _activation_as_crossing(level=-40.0):
    """Activation read as the first upward crossing of a fixed level."""
    def act(V_series, t_series):
        V, t = np.asarray(V_series), np.asarray(t_series)
        c = np.full(V.shape[1], -1.0)
        for n in range(len(t) - 1):
            c = ionic.threshold_crossing_update(c, V[n], V[n + 1], t[n], t[n + 1], level)
        return c, np.abs(np.diff(V, axis=0)).max(axis=0)
    return act


_ACT_PINS = [lambda: pins.test_activation_time_is_steepest_point_of_tanh_upstrokes(),
             lambda: pins.test_activation_time_ties_take_the_first_step()]
_VCYCLE_PINS = [lambda: pins.test_vcycle_coarse_correction_is_exact_on_a_constructed_hierarchy(3),
                lambda: pins.test_vcycle_beats_the_smoother_alone()]


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
    # V-cycle without its coarse-grid correction (smoothing only)
    "coarse correction dropped": (
        lambda mp: mp.setattr(solvers, "vcycle", _vcycle_with(correct=lambda x, Pxc: x)),
        _VCYCLE_PINS),
    # prolongated correction replaces the smoothed iterate instead of adding to it
    "prolongation not added": (
        lambda mp: mp.setattr(solvers, "vcycle", _vcycle_with(correct=lambda x, Pxc: Pxc)),
        _VCYCLE_PINS),
    # coarse correction scaled (a restriction weighted by 1/2, say)
    "coarse correction halved": (
        lambda mp: mp.setattr(solvers, "vcycle", _vcycle_with(correct=lambda x, Pxc: x + 0.5 * Pxc)),
        _VCYCLE_PINS),
    # the right-hand side restricted in place of the residual
    "restriction of b, not of the residual": (
        lambda mp: mp.setattr(solvers, "vcycle", _vcycle_with(restrict_residual=False)),
        _VCYCLE_PINS),
    # activation time as the first crossing of -40 mV instead of the steepest point
    "activation as a threshold crossing": (
        lambda mp: mp.setattr(ionic, "activation_times", _activation_as_crossing()),
        _ACT_PINS),
    # activation time stamped at the end of the steepest step, not its midpoint
    "activation stamped at step end": (
        lambda mp: mp.setattr(ionic, "activation_times", _activation_with(stamp="end")),
        _ACT_PINS),
    # signed derivative (a steep downstroke would not count)
    "activation without absolute value": (
        lambda mp: mp.setattr(ionic, "activation_times", _activation_with(absolute=False)),
        _ACT_PINS),
    # the later of two equally steep steps
    "activation ties to the last step": (
        lambda mp: mp.setattr(ionic, "activation_times", _activation_with(ties="last")),
        _ACT_PINS),
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
    """The same checks pass on the unmodified oracle (so a failure above is the mistake's),
    and the stand-ins used to plant mistakes reproduce the unmodified oracle."""
    for _, checks in MUTATIONS.values():
        for c in checks:
            c()
    import pytest as _pt
    mp = _pt.MonkeyPatch()
    try:
        mp.setattr(solvers, "vcycle", _vcycle_with())
        for c in _VCYCLE_PINS:
            c()
        mp.setattr(ionic, "activation_times", _activation_with())
        for c in _ACT_PINS:
            c()
    finally:
        mp.undo()
