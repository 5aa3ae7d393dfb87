"""GPU tests of the workflows around the hot path: autograd through apply and
solve (adjoint), the monodomain time loop, and parity at full workload sizes
(whole-vector parity on c2; sampled rows on the 51M-DOF p = 7 slab)."""
import functools

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import synth
from gpu_common import announce, rel_l2, to_dev, to_np
from oracle import adjoint as oadj
from oracle import ionic as oion
from oracle import operator as oop
from oracle import solvers as osol

pytestmark = pytest.mark.gpu

mf = pytest.importorskip("paper_2205_05136_amd")
from paper_2205_05136_amd import autograd as ag  # noqa: E402
from paper_2205_05136_amd import monodomain as md  # noqa: E402

GSPEC = synth.BoxSpec(p=3, n=(4, 3, 2), length=(2.0, 1.5, 1.0), fiber=True, theta0=-1.0,
                      theta1=1.0, sigma=synth.SLAB_SIGMA, alpha=28.0)


def test_apply_autograd_matches_oracle():
    announce("autograd apply")
    spec = GSPEC
    sig = synth.element_sigma(40, 2, spec.n_elem)
    box = mf.Box.from_spec(spec)
    op = mf.Operator.from_spec(spec, box=box, sigma=to_dev(sig))
    u = to_dev(synth.uniform(41, (2, spec.n_dof))).requires_grad_(True)
    w = synth.uniform(42, (2, spec.n_dof))
    s = to_dev(sig).requires_grad_(True)
    y = ag.apply(s, u, op)
    (y * to_dev(w)).sum().backward()
    for b in range(2):
        prob = oop.Problem(spec, sigma=sig[b])
        A, _, _ = prob.assemble()
        assert rel_l2(to_np(y)[b], A @ to_np(u)[b]) <= 1e-12
        assert rel_l2(to_np(u.grad)[b], A @ w[b]) <= 1e-12
        g_ref = oadj.grad_sigma(prob, to_np(u)[b], w[b])
        assert rel_l2(to_np(s.grad)[b], g_ref) <= 1e-12


def test_solve_adjoint_vs_oracle_and_finite_differences():
    announce("autograd solve + FD")
    spec = GSPEC
    sig = synth.element_sigma(43, 2, spec.n_elem)
    f = synth.uniform(44, (2, spec.n_dof))
    ut = 0.01 * synth.uniform(45, (2, spec.n_dof))
    solver = ag.Solver(spec, batch=2, rtol=1e-14, max_it=300)
    s = to_dev(sig).requires_grad_(True)
    fd_ = to_dev(f).requires_grad_(True)
    u = ag.solve(s, fd_, solver)
    L = 0.5 * ((u - to_dev(ut)) ** 2).sum()
    L.backward()
    g = to_np(s.grad)
    for b in range(2):
        prob = oop.Problem(spec, sigma=sig[b])
        Lb, g_ref, lam, u_ref = oadj.loss_and_grad(prob, f[b], ut[b])
        assert rel_l2(to_np(u)[b], u_ref) <= 1e-12
        assert rel_l2(g[b], g_ref) <= 1e-10
        assert rel_l2(to_np(fd_.grad)[b], lam) <= 1e-10

    def loss(sig_np):
        with torch.no_grad():
            uu = ag.solve(to_dev(sig_np), to_dev(f), solver)
            return 0.5 * float(((uu - to_dev(ut)) ** 2).sum())

    h = 1e-6
    for (b, e, c) in [(0, 0, 0), (0, 7, 1), (1, 13, 0), (1, 23, 1)]:
        sp_, sm_ = sig.copy(), sig.copy()
        sp_[b, e, c] += h
        sm_[b, e, c] -= h
        fd = (loss(sp_) - loss(sm_)) / (2 * h)
        assert abs(fd - g[b, e, c]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (b, e, c, fd, g[b, e, c])


def test_monodomain_steps_match_oracle():
    announce("monodomain 30 steps")
    spec = synth.slab(3, (6, 3, 2)).with_(length=(3.0, 1.5, 1.0))
    prm = synth.AP_PARAMS
    dt = 0.05
    stim = md.Stimulus(lo=(0, 0, 0), hi=(1.0, 1.0, 1.0), amplitude=50.0, duration=1.0)
    sim = md.Monodomain(spec, dt, synth.CHI, synth.CM, prm, stim, precision=torch.float64,
                        rtol=1e-14)
    # oracle: the same scheme with explicit matrices and direct solves
    ospec = spec.with_(alpha=synth.CHI * synth.CM / dt)
    prob = oop.Problem(ospec)
    A, M, _ = prob.assemble()
    m = M.diagonal()
    X = prob.mesh.xyz
    inside = np.all((X >= 0.0) & (X <= 1.0), axis=1)
    istim = inside * 50.0
    V = np.full(prob.n_dof, prm["v_rest"])
    w = np.zeros(prob.n_dof)
    Ainv = spla.factorized(A.tocsc())
    t = 0.0
    for n in range(30):
        b, w = oion.imex_rhs_and_gate(V, w, istim if t < 1.0 else 0.0 * istim, m, dt,
                                      synth.CHI, synth.CM, prm)
        V = Ainv(b)
        t += dt
        sim.step()
    assert V.max() > -70.0  # the stimulus has depolarised part of the slab
    assert rel_l2(to_np(sim.V), V) <= 1e-9
    assert rel_l2(to_np(sim.w), w) <= 1e-9


def test_c2_full_size_parity():
    announce("c2 full size apply + GMG-PCG")
    spec = synth.C2
    prob = oop.Problem(spec)
    A, _, _ = prob.assemble()
    ops, mg = mf.hierarchy(spec, coarsening=(("p", 2), ("p", 1)), degree=3)
    x = synth.uniform(100, spec.n_dof)
    assert rel_l2(to_np(ops[0].apply(to_dev(x))), A @ x) <= 1e-12
    f = synth.uniform(2, spec.n_dof)
    u, info = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-10, max_it=100)
    r = f - A @ to_np(u)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(f)
    # both sides solved to 1e-14: they agree within kappa(A) * 1e-14 (kappa < 100 here)
    u2, _ = mf.pcg(ops[0], to_dev(f), mg=mg, rtol=1e-14, max_it=100)
    x_ref, it, _ = osol.cg(A, f, rtol=1e-14)
    assert rel_l2(to_np(u2), x_ref) <= 1e-12


@functools.lru_cache(maxsize=4)
def _oracle_monodomain(spec, scheme, n_steps, dt, stim_lo, stim_hi, amp, dur):
    """The monodomain loop on the oracle: explicit matrices, direct solves, and
    the whole potential series (for the activation times)."""
    prm = synth.AP_PARAMS
    scale = 1.5 if scheme == "bdf2" else 1.0
    prob = oop.Problem(spec.with_(alpha=scale * synth.CHI * synth.CM / dt))
    A, M, _ = prob.assemble()
    m = M.diagonal()
    X = prob.mesh.xyz
    istim = np.all((X >= np.asarray(stim_lo)) & (X <= np.asarray(stim_hi)), axis=1) * amp
    V = np.full(prob.n_dof, prm["v_rest"])
    Vo, w, wo = V.copy(), np.zeros(prob.n_dof), np.zeros(prob.n_dof)
    Ainv = spla.factorized(A.tocsc())
    t, series, times = 0.0, [V.copy()], [0.0]
    for _ in range(n_steps):
        if scheme == "bdf2":
            on = t + dt <= dur
            b, w_new = oion.bdf2_rhs_and_gate(V, Vo, w, wo, istim if on else 0 * istim, m, dt,
                                              synth.CHI, synth.CM, prm)
            wo, w = w, w_new
        else:
            b, w = oion.imex_rhs_and_gate(V, w, istim if t < dur else 0 * istim, m, dt,
                                          synth.CHI, synth.CM, prm)
        Vo, V = V, Ainv(b)
        t += dt
        series.append(V.copy())
        times.append(t)
    return V, w, np.array(series), np.array(times)


def _check_activation(sim, series, times, dt, tol):
    """Activation times of the GPU loop against the oracle's (Section 5.1),
    computed with the oracle's running form from the same t and dt as the loop.
    The potentials agree to a relative l2 bar `tol`, so no node's value is off
    by more than e = tol ||V||_2 and no difference quotient by more than
    2e/dt.  Where the oracle's steepest step beats every other by more than
    twice that, the GPU's time must be that step's midpoint, to the bit (both
    compute t - dt/2 from the same t and dt); elsewhere (near ties) the GPU's
    step must be one whose oracle quotient is within 2e/dt of the steepest.
    The largest rates agree to the bar.  Returns the number of nodes of the
    first kind."""
    n = series.shape[1]
    tau, rate = np.full(n, -1.0), np.zeros(n)
    for k in range(len(times) - 1):
        tau, rate = oion.activation_update(tau, rate, series[k], series[k + 1], times[k + 1], dt)
    q = np.abs(np.diff(series, axis=0)) / dt
    a, r = to_np(sim.act), to_np(sim.act_rate)
    assert rel_l2(r, rate) <= tol
    eq = 2.0 * tol * np.linalg.norm(series[-1]) / dt
    top = np.sort(q, axis=0)
    margin = (top[-1] - top[-2]) > 2.0 * eq
    moved = rate > 0
    assert np.array_equal(a[margin & moved], tau[margin & moved])
    mid = times[1:] - 0.5 * dt
    for i in np.flatnonzero(~margin & moved):
        k = int(np.argmin(np.abs(mid - a[i])))
        assert mid[k] == a[i] and q[k, i] >= rate[i] - 2.0 * eq, i
    return int((margin & moved).sum())


def test_monodomain_bdf2_matches_oracle():
    """The paper's BDF2 partitioned scheme (Section 3), 60 steps from rest, with
    activation times (Section 5.1) and -40 mV crossings, against the oracle's
    direct solves."""
    announce("monodomain bdf2 60 steps")
    spec = synth.slab(3, (6, 3, 2)).with_(length=(3.0, 1.5, 1.0))
    dt, dur = 0.05, 2.0
    stim = md.Stimulus(lo=(0, 0, 0), hi=(1.0, 1.0, 1.0), amplitude=50.0, duration=dur)
    sim = md.Monodomain(spec, dt, synth.CHI, synth.CM, synth.AP_PARAMS, stim,
                        precision=torch.float64, rtol=1e-14, scheme="bdf2", v_cross=-40.0)
    V, w, series, times = _oracle_monodomain(spec, "bdf2", 60, dt, (0, 0, 0), (1.0, 1.0, 1.0),
                                             50.0, dur)
    for _ in range(60):
        sim.step()
    assert rel_l2(to_np(sim.V), V) <= 1e-9
    assert rel_l2(to_np(sim.w), w) <= 1e-9
    cross = np.full(V.size, -1.0)
    for k in range(60):
        cross = oion.threshold_crossing_update(cross, series[k], series[k + 1], times[k] ,
                                               times[k + 1], -40.0)
    assert (cross >= 0).sum() > 100  # part of the slab has activated
    c = to_np(sim.cross)
    assert np.array_equal(c < 0, cross < 0)
    assert np.max(np.abs(c[cross >= 0] - cross[cross >= 0])) <= 1e-6
    assert _check_activation(sim, series, times, dt, 1e-9) > V.size // 4
    # the steepest point of an upstroke comes after its -40 mV crossing
    up = (cross >= 0) & (series.max(axis=0) > 0.0)
    assert np.all(to_np(sim.act)[up] > c[up])


# The full monodomain workload (p = 5, p 5 -> 3 -> 1 multigrid with the FP32
# V-cycle inside FP64 flexible CG, 0.05 ms steps) at reduced size: 6 x 6 x 4
# elements at the workload's element edge (20/128 mm, the box 0.94 x 0.94 x
# 0.63 mm), fibers rotating -60..+60 degrees through the thickness, a 0.5 mm
# stimulated corner cube for the workload's 2 ms.
C5_SMALL = synth.C5.with_(n=(6, 6, 4), length=(6 * 20 / 128, 6 * 20 / 128, 4 * 10 / 64))


@pytest.mark.parametrize("scheme", ["imex1", "bdf2"])
@pytest.mark.parametrize("rtol,bar", [(1e-10, 1e-7), (1e-13, 1e-10)])
def test_c5_reduced_mixed_precision_loop(scheme, rtol, bar):
    """30 steps of the c5 loop in mixed precision against the oracle's FP64
    direct solves.  Bars: each solve stops at ||r|| <= rtol ||b|| (relative to
    the right-hand side, which the mass term dominates), so each step's error
    is at most kappa * rtol with kappa(A) < 30 here; the ionic update can
    amplify it near the upstroke, and 30 steps add up, so 1e3 * rtol."""
    announce(f"c5 reduced mixed {scheme} rtol={rtol}")
    spec, dt = C5_SMALL, 0.05
    stim = md.Stimulus(lo=(0, 0, 0), hi=(0.5, 0.5, 0.5), amplitude=50.0, duration=2.0)
    sim = md.Monodomain(spec, dt, synth.CHI, synth.CM, synth.AP_PARAMS, stim,
                        coarsening=(("p", 3), ("p", 1)), degree=3, precision=torch.float32,
                        rtol=rtol, scheme=scheme)
    V, w, series, times = _oracle_monodomain(spec, scheme, 30, dt, (0, 0, 0), (0.5,) * 3, 50.0, 2.0)
    for _ in range(30):
        info = sim.step()
        assert info.status == [0]
    assert series[-1].max() > -40.0  # the stimulus has depolarised part of the box
    e_v, e_w = rel_l2(to_np(sim.V), V), rel_l2(to_np(sim.w), w)
    print(f"c5 reduced {scheme} rtol {rtol}: V {e_v:.2e}, w {e_w:.2e}")
    assert e_v <= bar and e_w <= bar
    _check_activation(sim, series, times, dt, bar)


@pytest.mark.parametrize("p", [2, 4])
def test_full_size_properties(p):
    """At the 51M-DOF p-sweep size, properties that hold at any size: K
    annihilates constants (alpha = 0), A is symmetric (x^T A y = y^T A x), and
    1^T M 1 is the slab's volume 20 x 7 x 3 mm^3 (the shear keeps it)."""
    announce(f"full-size properties p{p}")
    spec = synth.sweep(p)
    op = mf.Operator.from_spec(spec, alpha=0.0)
    one = torch.ones(spec.n_dof, dtype=torch.float64, device="cuda")
    k1 = op.apply(one)
    g = torch.arange(spec.n_dof, device="cuda", dtype=torch.float64)
    x, y = torch.sin(0.37 * g), torch.cos(0.11 * g + 0.5)
    ax = op.apply(x)
    assert float(k1.abs().max()) <= 1e-12 * float(ax.abs().max())
    op.set_alpha(spec.alpha)
    ax, ay = op.apply(x), op.apply(y)
    xay, yax = float(torch.dot(x, ay)), float(torch.dot(y, ax))
    assert abs(xay - yax) <= 1e-12 * (float(torch.dot(x.abs(), ay.abs())) + 1.0)
    vol = float(op.apply_mass(one).sum())
    assert abs(vol - 420.0) <= 1e-9 * 420.0


FULL_SIZE = {"slab-p4-51M": synth.sweep(4), "slab-p7-51M": synth.C3_NI,
             "slab-p7-gauss-q9-51M": synth.C3_SEM,
             "slab-p4-gauss-51M": synth.sweep(4, quad="gauss", nq1d=6),
             "box-p5-132M": synth.C5}


@pytest.mark.parametrize("name", list(FULL_SIZE))
def test_full_size_sampled_rows(name):
    """At the workload sizes (51M and 132M DOFs), in the benchmark's launch
    configuration: rows of A x against the oracle's element matrices,
    x_g = sin(0.37 g); FP64 to 1e-12 and the FP32 kernel (FP32 G and vectors) to
    1e-5 of the rows' scale; and diagonal entries of the same rows."""
    announce(f"sampled rows {name}")
    spec = FULL_SIZE[name]
    op = mf.Operator.from_spec(spec, store_f32=True)
    g = torch.arange(spec.n_dof, device="cuda", dtype=torch.float64)
    x = torch.sin(0.37 * g)
    del g
    y = op.apply(x)
    y32 = op.apply(x.float())
    rng = np.random.default_rng(1)
    rows = np.concatenate([rng.integers(0, spec.n_dof, 24), [0, spec.n_dof - 1]])
    ref = oop.apply_rows(spec, lambda gg: np.sin(0.37 * np.asarray(gg, dtype=np.float64)), rows)
    idx = torch.as_tensor(rows, device="cuda")
    got, got32 = to_np(y[idx]), to_np(y32[idx])
    scale = np.abs(ref).max()
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale, (got - ref)
    assert np.max(np.abs(got32 - ref)) <= 1e-5 * scale, (got32 - ref)
    # diagonal entries A_gg of some of the rows (the row times the indicator of g)
    d, d32 = op.diagonal(), op.diagonal(torch.float32)
    for gg in rows[:6]:
        a_gg = oop.apply_rows(spec, lambda h: (np.asarray(h) == gg).astype(np.float64), [gg])[0]
        assert abs(float(d[int(gg)]) - a_gg) <= 1e-12 * abs(a_gg), (gg, float(d[int(gg)]), a_gg)
        assert abs(float(d32[int(gg)]) - a_gg) <= 1e-5 * abs(a_gg), (gg, float(d32[int(gg)]), a_gg)


def test_c4_full_size_batch_sampled_rows():
    """c4 at full size as the benchmark launches it: one apply over the batch of 8
    per-element conductivity sets (8 x 2,146,689 DOFs); sampled rows of every
    member against the oracle's element matrices with that member's sigma, FP64
    to 1e-12 and FP32 to 1e-5 of the rows' scale."""
    announce("c4 full-size batch sampled rows")
    spec = synth.C4
    B = 8
    sig = synth.element_sigma(4, B, spec.n_elem)
    op = mf.Operator.from_spec(spec, sigma=to_dev(sig), store_f32=True)
    g = torch.arange(spec.n_dof, device="cuda", dtype=torch.float64)
    x = torch.stack([torch.sin(0.37 * g + 0.1 * b) for b in range(B)]).contiguous()
    y, y32 = op.apply(x), op.apply(x.float())
    rng = np.random.default_rng(2)
    for b in range(B):
        rows = np.concatenate([rng.integers(0, spec.n_dof, 6), [0, spec.n_dof - 1]])
        ref = oop.apply_rows(
            spec, lambda gg: np.sin(0.37 * np.asarray(gg, dtype=np.float64) + 0.1 * b), rows,
            sigma=sig[b])
        idx = torch.as_tensor(rows, device="cuda")
        got, got32 = to_np(y[b][idx]), to_np(y32[b][idx])
        scale = np.abs(ref).max()
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale, (b, got - ref)
        assert np.max(np.abs(got32 - ref)) <= 1e-5 * scale, (b, got32 - ref)


def test_c4_full_size_batch_grad_sampled_elements():
    """The dL/dsigma contraction g[e, c] = w^T (dA/dsigma_{e,c}) u at the c4 size for
    the batch of 8, as the benchmark's backward pass runs it; sampled elements of
    every member against the oracle's explicit dK_e (which do not depend on sigma,
    A being linear in it), to 1e-12 of the sampled entries' scale."""
    announce("c4 full-size batch gradient, sampled elements")
    spec = synth.C4
    B = 8
    sig = synth.element_sigma(4, B, spec.n_elem)
    op = mf.Operator.from_spec(spec, sigma=to_dev(sig))
    g = torch.arange(spec.n_dof, device="cuda", dtype=torch.float64)
    u = torch.stack([torch.sin(0.37 * g + 0.1 * b) for b in range(B)]).contiguous()
    w = torch.stack([torch.cos(0.23 * g + 0.2 * b) for b in range(B)]).contiguous()
    grad = to_np(op.grad_sigma(u, w)).reshape(B, spec.n_elem, 3)
    prob = oop.Problem(spec)
    rng = np.random.default_rng(3)
    els = np.concatenate([rng.integers(0, spec.n_elem, 14), [0, spec.n_elem - 1]])
    _, _, dK = prob.elem_matrices(els, parts=True)
    ed = prob.elem_dof[els]
    for b in range(B):
        ub = np.sin(0.37 * ed.astype(np.float64) + 0.1 * b)
        wb = np.cos(0.23 * ed.astype(np.float64) + 0.2 * b)
        ref = np.einsum("ceij,ei,ej->ec", dK, wb, ub)
        got = grad[b][els]
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(ref).max(), (b, got - ref)


# the benchmark's solves at full size: its default workload (p = 4), the p-sweep's
# ends and c3 (GLL and Gauss), each with the benchmark's degree chain
FULL_SOLVES = {"slab-p4-51M": (synth.sweep(4), (("p", 2), ("p", 1))),
               "slab-p2-51M": (synth.sweep(2), (("p", 1),)),
               "slab-p4-gauss-51M": (synth.sweep(4, quad="gauss", nq1d=6), (("p", 2), ("p", 1))),
               "c3-gll-q8": (synth.C3_NI, (("p", 5), ("p", 3), ("p", 1))),
               "c3-gauss-q9": (synth.C3_SEM, (("p", 5), ("p", 3), ("p", 1)))}


@pytest.mark.parametrize("name", list(FULL_SOLVES))
def test_full_size_solve_certificate(name):
    """The benchmark's solves at full size (about 51M DOFs): the FP64 and the
    mixed-precision solves to 1e-10, certified against the oracle where it
    cannot solve.  On sampled rows, b - A x with the oracle's element matrices
    (i) stays within 10x the per-row RMS the tolerance allows,
    1e-10 ||b|| / sqrt(N), and (ii) equals the GPU's own true residual, which
    is within the tolerance over the whole vector, to 1e-11 max|b|: x is about
    1e3 times larger than b here (the mass term dominates and the elements are
    small), so each row cancels stiffness terms of order 1e2 |b| summed over up
    to 4096 products, and FP64 rounding of those terms is ~1e-12 |b|.  The two
    solutions agree to 1e-8."""
    announce(f"full-size solve certificate {name}")
    spec, chain = FULL_SOLVES[name]
    f = torch.as_tensor(synth.uniform(3, spec.n_dof), device="cuda")
    rng = np.random.default_rng(3)
    rows = np.concatenate([rng.integers(0, spec.n_dof, 16), [0, spec.n_dof - 1]])
    trow = torch.as_tensor(rows, device="cuda")
    fmax, fnorm = float(f.abs().max()), float(torch.linalg.norm(f))
    sols = {}
    for precision in (torch.float64, torch.float32):
        ops, mg = mf.hierarchy(spec, coarsening=chain, degree=3, precision=precision)
        x, info = mf.pcg(ops[0], f, mg=mg, rtol=1e-10, max_it=100)
        assert info.status == [0], info
        r = f - ops[0].apply(x)
        assert float(torch.linalg.norm(r)) <= 1.01e-10 * fnorm
        xh = to_np(x)
        ax_ref = oop.apply_rows(spec, lambda g: xh[np.asarray(g)], rows)
        r_ref = to_np(f[trow]) - ax_ref
        print(f"{spec.quad} {precision}: oracle rows |r| max {np.abs(r_ref).max():.2e}, "
              f"vs GPU residual {np.abs(r_ref - to_np(r[trow])).max():.2e}")
        assert np.abs(r_ref).max() <= 10 * 1e-10 * fnorm / np.sqrt(spec.n_dof), precision
        assert np.max(np.abs(r_ref - to_np(r[trow]))) <= 1e-11 * fmax, precision
        sols[precision] = x
        del ops, mg
    assert rel_l2(to_np(sols[torch.float32]), to_np(sols[torch.float64])) <= 1e-8


def test_extrapolated_guess_gives_the_same_steps():
    """The initial guess 2 V^n - V^{n-1} (mfsem_extrapolate, exact elementwise)
    changes only the iterations of each solve, not the time steps."""
    announce("extrapolated initial guess")
    v = synth.uniform(60, 1000)
    vo = synth.uniform(61, 1000)
    out = to_np(mf.extrapolate(to_dev(v), to_dev(vo)))
    assert np.array_equal(out, 2.0 * v - vo)
    spec = synth.slab(3, (6, 3, 2)).with_(length=(3.0, 1.5, 1.0))
    stim = md.Stimulus(lo=(0, 0, 0), hi=(1.0, 1.0, 1.0), amplitude=50.0, duration=1.0)
    runs = {}
    for guess in ("extrapolate", "previous"):
        sim = md.Monodomain(spec, 0.05, synth.CHI, synth.CM, synth.AP_PARAMS, stim,
                            precision=torch.float64, rtol=1e-13, scheme="bdf2", guess=guess)
        its = [sim.step().iters[0] for _ in range(30)]
        runs[guess] = (to_np(sim.V), sum(its))
    assert rel_l2(runs["extrapolate"][0], runs["previous"][0]) <= 1e-10
    assert runs["extrapolate"][1] < runs["previous"][1], runs
