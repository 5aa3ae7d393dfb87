"""Full monodomain time loop: the outer loop of Alg. 1 around the hot path.

Per step (first-order IMEX; the paper's scheme is BDF2 with extrapolation,
Section 3): the pointwise Aliev-Panfilov update and SEM-NI right-hand side
(mfsem_ap_imex_rhs), then (alpha M + K) V^{n+1} = b by GMG-PCG warm-started from
V^n (Section 5), alpha = chi Cm / dt.  All arithmetic runs in libmfsem.
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
                 rtol=1e-10, atol=0.0, device="cuda"):
        self.spec = spec.with_(alpha=chi * cm / dt)
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
        self.t = 0.0
        self.stats = StepStats()

    def step(self):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        stim = self.i_stim if self.t < self.stim.duration else None
        api.ap_imex_rhs(self.V, self.w, self.mass, self.dt, self.chi, self.cm, self.prm,
                        i_stim=stim, out=self.b)
        ev[1].record()
        V, info = api.pcg(self.op, self.b, x0=self.V, mg=self.mg, rtol=self.rtol, atol=self.atol,
                          max_it=500)
        ev[2].record()
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
