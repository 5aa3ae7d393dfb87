"""Pointwise ionic step and right-hand side for the full monodomain workload.

The paper's ionic models (TTP06, CRN) are only cited; the workload uses the
two-variable Aliev-Panfilov model in its place.  With u = (V - v_rest)/v_amp
and tau = t / t_scale:

    du/dtau = F(u, w) = k u (1 - u)(u - a) - u w
    dw/dtau = eps(u, w) (-w - k u (u - a - 1)),  eps = eps0 + mu1 w / (u + mu2)

First-order IMEX step of chi Cm dV/dt = div(sigma grad V) + chi Cm (v_amp/t_scale) F + I_stim
(Section 3 writes the BDF2 version of this splitting; the ionic terms are taken
explicitly at V^n):

    w^{n+1} = w^n + (dt/t_scale) eps (-w^n - k u^n (u^n - a - 1))
    (alpha M + K) V^{n+1} = M (alpha V^n + chi Cm (v_amp/t_scale) F(u^n, w^n) + I_stim),
    alpha = chi Cm / dt,

where M is the (diagonal, SEM-NI) mass matrix, so the right-hand side is
pointwise: b_i = M_ii * (...)_i.
"""
from __future__ import annotations

import numpy as np


def ap_rates(u, w, k, a, eps0, mu1, mu2, **_):
    F = k * u * (1.0 - u) * (u - a) - u * w
    eps = eps0 + mu1 * w / (u + mu2)
    G = eps * (-w - k * u * (u - a - 1.0))
    return F, G


def imex_rhs_and_gate(V, w, i_stim, mass_diag, dt, chi, cm, prm):
    """Returns (b, w_next) for one step, elementwise loops written with numpy."""
    u = (V - prm["v_rest"]) / prm["v_amp"]
    F, G = ap_rates(u, w, **prm)
    alpha = chi * cm / dt
    b = mass_diag * (alpha * V + chi * cm * (prm["v_amp"] / prm["t_scale"]) * F + i_stim)
    w_next = w + (dt / prm["t_scale"]) * G
    return b, w_next


# --- BDF2 partitioned scheme (Section 3, the ionic and monodomain discretization) ---
#
# Gating, implicit in w^{n+1} with the extrapolated potential V* = 2 V^n - V^{n-1}:
#     (3 w^{n+1} - 4 w^n + w^{n-1}) / (2 dt) = G(u*, w^{n+1}) / t_scale
# Potential: (3 alpha1/2 M + K) V^{n+1} = M (alpha1 (4 V^n - V^{n-1}) / 2
#            + chi Cm (v_amp/t_scale) F(u*, w^{n+1}) + I_stim),  alpha1 = chi Cm / dt,
# with the ionic current taken at (V*, w^{n+1}) (ionic current interpolation,
# which for SEM-NI is the lumped form, so the right-hand side is pointwise).

def bdf2_gate(u_star, w_n, w_nm1, dt, k, a, eps0, mu1, mu2, t_scale, iters=60, **_):
    """w^{n+1} solving the scalar BDF2 gating equation at every DOF, by Newton's
    method on R(w) = 3w - 4w^n + w^{n-1} - (2 dt / t_scale) G(u*, w), started at
    the BDF1 predictor and run to convergence (R is quadratic in w)."""
    h = 2.0 * dt / t_scale
    w = np.array(w_n, dtype=np.float64, copy=True)
    c = k * u_star * (u_star - a - 1.0)
    r = mu1 / (u_star + mu2)
    for _ in range(iters):
        G = (eps0 + r * w) * (-w - c)
        dG = r * (-w - c) - (eps0 + r * w)
        R = 3.0 * w - 4.0 * w_n + w_nm1 - h * G
        dR = 3.0 - h * dG
        step = R / dR
        w = w - step
        if np.all(np.abs(step) <= 1e-16 * np.maximum(1.0, np.abs(w))):
            break
    return w


def bdf2_rhs_and_gate(V, V_old, w, w_old, i_stim, mass_diag, dt, chi, cm, prm):
    """Returns (b, w_next) of one BDF2 step: the gating update and the pointwise
    right-hand side of (3/2 alpha1 M + K) V^{n+1} = b."""
    V_star = 2.0 * V - V_old
    u_star = (V_star - prm["v_rest"]) / prm["v_amp"]
    w_next = bdf2_gate(u_star, w, w_old, dt, **prm)
    F, _ = ap_rates(u_star, w_next, **prm)
    alpha1 = chi * cm / dt
    b = mass_diag * (alpha1 * (4.0 * V - V_old) / 2.0
                     + chi * cm * (prm["v_amp"] / prm["t_scale"]) * F + i_stim)
    return b, w_next


def activation_times(V_series, t_series):
    """Activation time at every DOF from a whole time series (Section 5.1, the
    activation-time definition: the instant at which the potential changes
    fastest, tau(x_i) = argmax_t |du/dt(x_i, t)|).

    V_series [n_steps+1][n_dof] holds V at the times t_series [n_steps+1].  The
    derivative over step n is the difference quotient (V^{n+1} - V^n) /
    (t^{n+1} - t^n), a second-order estimate of du/dt at the step's midpoint,
    so tau is that midpoint for the step with the largest |quotient|; on ties
    the earliest step wins.  A DOF whose potential never changes keeps -1.
    Returns (tau, largest |du/dt|)."""
    V = np.asarray(V_series, dtype=np.float64)
    t = np.asarray(t_series, dtype=np.float64)
    n_dof = V.shape[1]
    tau = np.full(n_dof, -1.0)
    rate = np.zeros(n_dof)
    for i in range(n_dof):
        for n in range(len(t) - 1):
            dt = t[n + 1] - t[n]
            r = abs(V[n + 1, i] - V[n, i]) / dt
            if r > rate[i]:
                rate[i] = r
                tau[i] = t[n + 1] - 0.5 * dt
    return tau, rate


def activation_update(act, rate, V_old, V, t, dt):
    """The same definition kept as a running maximum, one step at a time (the
    form a time loop can afford), for a step from V_old at t - dt to V at t:
    where |V - V_old| / dt exceeds rate, rate takes it and act the step's
    midpoint t - dt/2.  Start from act = -1 and rate = 0; after the last step
    act equals activation_times over the series.  Returns new (act, rate)."""
    act = np.array(act, dtype=np.float64, copy=True)
    rate = np.array(rate, dtype=np.float64, copy=True)
    for i in range(len(act)):
        r = abs(V[i] - V_old[i]) / dt
        if r > rate[i]:
            rate[i] = r
            act[i] = t - 0.5 * dt
    return act, rate


def threshold_crossing_update(cross, V_old, V, t_old, t_new, v_cross):
    """First upward crossing of the level v_cross at every DOF, linearly
    interpolated in time between two steps; cross < 0 marks 'not yet'.  Not the
    paper's activation time (which is the steepest point of the upstroke, later
    than a crossing below it); kept as a separately named output."""
    cross = np.array(cross, dtype=np.float64, copy=True)
    for i in range(len(cross)):
        if cross[i] < 0.0 and V_old[i] < v_cross <= V[i]:
            cross[i] = t_old + (t_new - t_old) * (v_cross - V_old[i]) / (V[i] - V_old[i])
    return cross
