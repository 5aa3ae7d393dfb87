"""The appendix's BDF1/2/3 heat-equation study (tests/heat_bdf.py), on the
oracle (CPU) and through the library (GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from heat_bdf import BDF, run
from oracle import operator as oop

CUBE = synth.BoxSpec(p=3, n=(2, 2, 2))  # unit cube, h = 0.5, sigma = 1


def _oracle_errors(spec, kind, order, dts, T=1.0):
    errs = []
    for dt in dts:
        a0 = BDF[order][0]
        prob = oop.Problem(spec.with_(alpha=a0 / dt))
        A, M, _ = prob.assemble()
        solve = spla.factorized(A.tocsc())
        errs.append(run(kind, order, dt, T, prob.mesh.xyz, M.diagonal(), solve))
    return np.array(errs)


@pytest.mark.parametrize("p", [3, 4])
def test_bdf_orders_on_a_solution_exact_in_space(p):
    """Q_p (p >= 3) holds the cubic solution exactly: BDF-k converges at order k."""
    spec = CUBE.with_(p=p)
    dts = [0.02, 0.01, 0.005]
    for order in (1, 2, 3):
        e = _oracle_errors(spec, "poly", order, dts)
        rates = np.log2(e[:-1] / e[1:])
        assert np.all(np.abs(rates - order) < 0.1), (order, e, rates)


def test_space_error_floor_makes_bdf3_no_better():
    """On a solution Q_3 misses, the error stops at the space error: at small dt
    BDF2 and BDF3 reach the same floor, far below BDF1 (the appendix's point)."""
    dts = [0.02]
    e1 = _oracle_errors(CUBE, "trig", 1, dts)[0]
    e2 = _oracle_errors(CUBE, "trig", 2, dts)[0]
    e3 = _oracle_errors(CUBE, "trig", 3, dts)[0]
    assert abs(e2 - e3) < 0.05 * e3, (e1, e2, e3)
    assert e1 > 1.5 * e2, (e1, e2, e3)


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["poly", "trig"])
def test_bdf_study_through_the_library(kind):
    """The same study with the library's operator (alpha = a0/dt), mass and PCG:
    the errors agree with the oracle's."""
    mf = pytest.importorskip("paper_2205_05136_amd")
    import torch
    from gpu_common import announce, to_dev, to_np
    announce(f"heat BDF study {kind}")
    dt = 0.01
    for order in (1, 2, 3):
        op = mf.Operator.from_spec(CUBE.with_(alpha=BDF[order][0] / dt))
        mass = to_np(op.apply_mass(torch.ones(op.n_dof, dtype=torch.float64, device="cuda")))
        xyz = to_np(op.geometry.xyz)
        solve = lambda rhs: to_np(mf.pcg(op, to_dev(rhs), rtol=1e-14, max_it=2000)[0])
        e_gpu = run(kind, order, dt, 1.0, xyz, mass, solve)
        e_orc = _oracle_errors(CUBE, kind, order, [dt])[0]
        assert abs(e_gpu - e_orc) <= 1e-6 * e_orc, (order, e_gpu, e_orc)
