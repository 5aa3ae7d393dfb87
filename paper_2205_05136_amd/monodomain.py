"""Full monodomain time loop: the outer loop of Alg. 1 around the hot path.

Two schemes, both a pointwise ionic update and SEM-NI right-hand side followed
by one GMG-PCG solve, warm-started (Section 5) from the extrapolation
2 V^n - V^{n-1} (guess="extrapolate", about a quarter fewer iterations) or
from V^n (guess="previous"):
  "imex1": first-order IMEX (mfsem_ap_imex_rhs), (alpha M + K) V^{n+1} = b with
           alpha = chi Cm / dt;
  "bdf2":  the paper's partitioned BDF2 scheme (Section 3) with the
           extrapolation V* = 2 V^n - V^{n-1}, the gating equation implicit in
           w^{n+1} and the ionic current at (V*, w^{n+1}) (mfsem_ap_bdf2_rhs),
           (3/2 alpha M + K) V^{n+1} = b; the first step starts from rest
           (V^{-1} = V^0, w^{-1} = w^0).
After every solve the activation time of each DOF (Section 5.1: the time of
the largest |dV/dt|, the midpoint of the steepest step; -1 while V has not
moved) and the largest |dV/dt| are updated (mfsem_activation_update), and,
if v_cross is given, the first upward crossing of that level.
All arithmetic runs in libmfsem.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from . import api


@dataclass
class Stimulus:
    lo: tuple             # box corner [mm]
    hi: tuple             # opposite corner [mm]
    amplitude: float      # uA/mm^3
    duration: float       # ms


@dataclass
class StepStats:
    iters: list = field(default_factory=list)
    solve_ms: list = field(default_factory=list)
    ionic_ms: list = field(default_factory=list)


class Monodomain:
    def __init__(self, spec, dt, chi, cm, ap_params: dict, stimulus: Stimulus,
                 coarsening=(("p", 2), ("p", 1)), degree=3, precision=torch.float32,
                 rtol=1e-10, atol=0.0, device="cuda", scheme="imex1", v_cross=None,
                 guess="extrapolate"):
        if scheme not in ("imex1", "bdf2"):
            raise ValueError("scheme must be 'imex1' or 'bdf2'")
        if guess not in ("extrapolate", "previous"):
            raise ValueError("guess must be 'extrapolate' or 'previous'")
        # initial guess of each solve: 2 V^n - V^{n-1} (the scheme's V*), or V^n
        self.guess = guess
        self.scheme = scheme
        self.v_cross = None if v_cross is None else float(v_cross)
        scale = 1.5 if scheme == "bdf2" else 1.0
        self.spec = spec.with_(alpha=scale * chi * cm / dt)
        self.dt, self.chi, self.cm, self.prm = dt, chi, cm, ap_params
        self.rtol, self.atol = rtol, atol
        self.ops, self.mg = api.hierarchy(self.spec, coarsening=coarsening, degree=degree,
                                          precision=precision, device=device)
        op = self.ops[0]
        self.op = op
        ones = torch.ones(op.n_dof, dtype=torch.float64, device=op.device)
        self.mass = op.apply_mass(ones)  # the diagonal SEM-NI mass
        xyz = op.geometry.xyz
        inside = torch.ones(op.n_dof, dtype=torch.bool, device=op.device)
        for d in range(3):
            inside &= (xyz[:, d] >= stimulus.lo[d]) & (xyz[:, d] <= stimulus.hi[d])
        self.i_stim = inside.double() * stimulus.amplitude
        self.stim = stimulus
        self.V = torch.full((op.n_dof,), float(ap_params["v_rest"]), dtype=torch.float64,
                            device=op.device)
        self.w = torch.zeros_like(self.V)
        self.b = torch.empty_like(self.V)
        # BDF2 history (start from rest); activation times (-1: V has not moved),
        # the steepest rate so far, and level crossings (-1: not yet)
        self.V_old = self.V.clone()
        self.w_old = self.w.clone()
        self.act = torch.full_like(self.V, -1.0)
        self.act_rate = torch.zeros_like(self.V)
        self.cross = None if v_cross is None else torch.full_like(self.V, -1.0)
        self.t = 0.0
        self.stats = StepStats()

    def step(self):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        if self.scheme == "imex1":
            stim = self.i_stim if self.t < self.stim.duration else None
            api.ap_imex_rhs(self.V, self.w, self.mass, self.dt, self.chi, self.cm, self.prm,
                            i_stim=stim, out=self.b)
        else:
            # the applied current at t^{n+1}
            stim = self.i_stim if self.t + self.dt <= self.stim.duration else None
            api.ap_bdf2_rhs(self.V, self.V_old, self.w, self.w_old, self.mass, self.dt, self.chi,
                            self.cm, self.prm, i_stim=stim, out=self.b)
        ev[1].record()
        x0 = api.extrapolate(self.V, self.V_old) if self.guess == "extrapolate" else self.V
        V, info = api.pcg(self.op, self.b, x0=x0, mg=self.mg, rtol=self.rtol, atol=self.atol,
                          max_it=500)
        api.activation_update(V, self.V, self.t + self.dt, self.dt, act=self.act,
                              rate=self.act_rate, v_cross=self.v_cross or 0.0, cross=self.cross)
        ev[2].record()
        self.V_old = self.V
        self.V = V
        self.t += self.dt
        torch.cuda.synchronize()
        self.stats.iters.append(info.iters[0])
        self.stats.ionic_ms.append(ev[0].elapsed_time(ev[1]))
        self.stats.solve_ms.append(ev[1].elapsed_time(ev[2]))
        return info

    def run(self, n_steps):
        for _ in range(n_steps):
            self.step()
        return self.V
