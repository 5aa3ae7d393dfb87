"""Convergence of the GPU path on a manufactured solution (Section 3: the error of
the degree-p spectral element solution decays like h^{p+1} in the mass norm and
faster than any power of 1/p), at mesh sizes the oracle does not reach.

alpha u - div(grad u) = f on a warped unit cube with u = cos(pi x) cos(pi y)
cos(pi z), whose normal derivative vanishes on the faces (the natural boundary
condition of the operator).  The load vector is the mass matrix applied to the
nodal values of f: with GLL collocation this is exactly the quadrature of
f phi_i; with Gauss quadrature it is the consistent mass of the interpolant of f,
whose error is of the same order h^{p+1} as the one under test.  Nothing here
comes from the oracle: the checks are rates the mathematics fixes.  (The nodal
error measured here converges faster than the bound, close to h^{p+2} at
p = 2..4; only the bound is asserted.)"""
import math

import numpy as np
import pytest
import torch

import synth
from gpu_common import announce, to_dev

pytestmark = pytest.mark.gpu

mf = pytest.importorskip("paper_2205_05136_amd")

ALPHA = 1.0


def _warp(xyz, eps=0.04):
    """Interior warping that keeps the unit cube's faces in place."""
    s = np.sin(np.pi * xyz[:, 0]) * np.sin(np.pi * xyz[:, 1]) * np.sin(np.pi * xyz[:, 2])
    return eps * np.stack([s, 0.7 * s, -0.5 * s], axis=1)


def _problem(p, n, quad="gll", q=0, aniso=False):
    """aniso: fibers along x with sigma_l = 2, sigma_t = 0.5, i.e. sigma =
    diag(2, 0.5, 0.5); the normal flux sigma grad u . n still vanishes on the
    faces and -div(sigma grad u) = pi^2 (2 + 0.5 + 0.5) u."""
    sig = (2.0, 0.5, 0.5) if aniso else (1.0, 1.0, 1.0)
    spec = synth.BoxSpec(p=p, n=(n, n, n), quad=quad, nq1d=q, alpha=ALPHA, sigma=sig,
                         fiber=aniso)
    box = mf.Box.from_spec(spec)
    X = box.xyz.cpu().numpy()
    X = X + _warp(X)
    op = mf.Operator.from_spec(spec, box=box, xyz=to_dev(X))
    u_ex = np.cos(np.pi * X[:, 0]) * np.cos(np.pi * X[:, 1]) * np.cos(np.pi * X[:, 2])
    b = op.apply_mass(to_dev((ALPHA + np.pi ** 2 * sum(sig)) * u_ex))
    return spec, box, X, op, to_dev(u_ex), b


def _mass_norm(op, e):
    return math.sqrt(float(torch.dot(e, op.apply_mass(e))))


def _chain(p):
    pc = max(1, p // 2)
    return (("p", pc), ("p", 1)) if pc > 1 else (("p", 1),)


def _solve(spec, box, X, b, precision=torch.float64):
    """GMG-PCG whose p-levels keep the fine level's warped map."""
    ops, mg = mf.hierarchy(spec, fine_box=box, xyz=to_dev(X), coarsening=_chain(spec.p),
                           precision=precision, degree=3)
    u, info = mf.pcg(ops[0], b, mg=mg, rtol=1e-13, max_it=300)
    assert info.status == [0], (spec.p, spec.n, precision, info)
    return u, info


def _error(p, n, quad="gll", q=0, aniso=False):
    spec, box, X, op, u_ex, b = _problem(p, n, quad, q, aniso)
    u, _ = _solve(spec, box, X, b)
    return _mass_norm(op, u - u_ex)


@pytest.mark.parametrize("p,quad,q,aniso", [(2, "gll", 0, False), (3, "gll", 0, False),
                                            (4, "gll", 0, False), (3, "gauss", 5, False),
                                            (3, "gll", 0, True), (3, "gauss", 5, True)])
def test_h_convergence_rate(p, quad, q, aniso):
    announce(f"h-convergence p={p} {quad} aniso={aniso}")
    ns = (4, 8, 16)
    errs = [_error(p, n, quad, q, aniso) for n in ns]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    print(f"p = {p} {quad} aniso={aniso}: errors {errs}, rates {rates}", flush=True)
    # the finest pair is in the asymptotic range; the coarse pair may not be yet
    assert rates[-1] > p + 1 - 0.3, (errs, rates)
    assert rates[0] > p + 1 - 1.0, (errs, rates)


def test_p_convergence_is_faster_than_algebraic():
    announce("p-convergence n=4")
    errs = [_error(p, 4) for p in range(2, 8)]
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    print(f"p = 2..7 errors {errs}, ratios {ratios}", flush=True)
    assert all(r > 4 for r in ratios), (errs, ratios)


def test_mixed_precision_solve_reaches_the_same_discretisation_error():
    """The FP32 V-cycle inside flexible FP64 CG reaches the discretisation error of
    the FP64 GMG-PCG (warped fine level, p-levels 4 -> 2 -> 1 on the same map)."""
    announce("manufactured solution, GMG-PCG FP64 and mixed")
    spec, box, X, op, u_ex, b = _problem(4, 16)
    u64, info64 = _solve(spec, box, X, b)
    u32, info32 = _solve(spec, box, X, b, torch.float32)
    assert info64.iters[0] <= 40 and info32.iters[0] <= 40, (info64, info32)
    e64, e32 = _mass_norm(op, u64 - u_ex), _mass_norm(op, u32 - u_ex)
    print(f"errors FP64 {e64} ({info64.iters[0]} it), mixed {e32} ({info32.iters[0]} it)",
          flush=True)
    assert abs(e32 - e64) <= 1e-6 * e64, (e32, e64)
    assert _mass_norm(op, u32 - u64) <= 1e-8 * _mass_norm(op, u64)
