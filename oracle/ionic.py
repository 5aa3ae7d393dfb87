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
