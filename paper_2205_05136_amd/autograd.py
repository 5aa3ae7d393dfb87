"""torch.autograd Functions over the operator and its solve.

The operator A(sigma) = alpha M + K(sigma) is linear in every element's
conductivities sigma_e = (sigma_l, sigma_t, sigma_n) (Section 2, the diffusion
tensor), and symmetric.  Hence:

  y = A(sigma) u:        dL/du = A ybar,     dL/dsigma_e = ybar^T (dA/dsigma_e) u
  u = A(sigma)^{-1} f:   A lam = ubar,       dL/df = lam,   dL/dsigma_e = -lam^T (dA/dsigma_e) u

The backward of the solve is one more preconditioned CG solve (the adjoint
system is the same matrix); no CG iterate of the forward solve is stored.
The contractions w^T (dA/dsigma_e) u run in mfsem_op_grad_sigma.
"""
from __future__ import annotations

import torch

from . import api


class ApplyFn(torch.autograd.Function):
    """y = A(sigma) u with op built for per-element sigma ([batch][n_elem][3])."""

    @staticmethod
    def forward(ctx, sigma, u, op: api.Operator):
        op.set_sigma(sigma.detach())
        shape = u.shape
        y = op.apply(u.detach().contiguous().reshape(-1)).reshape(shape)
        ctx.op = op
        ctx.save_for_backward(sigma.detach(), u.detach())
        return y

    @staticmethod
    def backward(ctx, ybar):
        sigma, u = ctx.saved_tensors
        op = ctx.op
        op.set_sigma(sigma)
        yb = ybar.contiguous().reshape(-1)
        du = op.apply(yb).reshape(u.shape) if ctx.needs_input_grad[1] else None
        dsig = None
        if ctx.needs_input_grad[0]:
            dsig = op.grad_sigma(u.reshape(-1), yb).reshape(sigma.shape)
        return dsig, du, None


class Solver:
    """A(sigma) u = f by GMG-PCG on a structured box, rebuilt when sigma changes.

    spec: synth.BoxSpec; batch members solve independently in one set of launches."""

    def __init__(self, spec, batch=1, coarsening=(("p", 2), ("p", 1)), degree=3, rtol=1e-12,
                 max_it=500, precision=torch.float64, device="cuda"):
        self.spec, self.batch, self.coarsening = spec, batch, coarsening
        self.degree, self.rtol, self.max_it, self.precision = degree, rtol, max_it, precision
        self.box = api.Box.from_spec(spec, device=device)
        self.device = self.box.device
        self.sigma = None
        self.ops = self.mg = None

    def set_sigma(self, sigma):
        sigma = sigma.detach().to(self.device, torch.float64).contiguous()
        if self.sigma is not None and torch.equal(sigma, self.sigma):
            return
        self.sigma = sigma
        self.ops, self.mg = api.hierarchy(self.spec, fine_box=self.box, coarsening=self.coarsening,
                                          precision=self.precision, sigma=sigma,
                                          degree=self.degree)

    def solve(self, f):
        u, info = api.pcg(self.ops[0], f.contiguous().reshape(-1), mg=self.mg, rtol=self.rtol,
                          max_it=self.max_it)
        return u.reshape(f.shape), info


class SolveFn(torch.autograd.Function):
    """u = A(sigma)^{-1} f."""

    @staticmethod
    def forward(ctx, sigma, f, solver: Solver):
        solver.set_sigma(sigma)
        u, _ = solver.solve(f.detach())
        ctx.solver = solver
        ctx.save_for_backward(sigma.detach(), u)
        return u

    @staticmethod
    def backward(ctx, ubar):
        sigma, u = ctx.saved_tensors
        s = ctx.solver
        s.set_sigma(sigma)
        lam, _ = s.solve(ubar.detach())  # adjoint solve: A is symmetric
        dsig = None
        if ctx.needs_input_grad[0]:
            # dL/dsigma_e = -lam^T (dA/dsigma_e) u: the library applies the sign
            dsig = s.ops[0].grad_sigma(u.reshape(-1), lam.reshape(-1), scale=-1.0).reshape(
                sigma.shape)
        df = lam if ctx.needs_input_grad[1] else None
        return dsig, df, None


def apply(sigma, u, op):
    return ApplyFn.apply(sigma, u, op)


def solve(sigma, f, solver):
    return SolveFn.apply(sigma, f, solver)
