"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds workload parameters and random draws only.  None of the
method's arithmetic lives here: no quadrature, no Lagrange bases, no node
placement, no geometry and no operator.  Each side (the CPU oracle and the HIP
library) turns a `BoxSpec` into a mesh with its own code.

Random numbers come from `torch.Generator().manual_seed(seed)` on the CPU in
float64, so every consumer sees bit-identical inputs.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np
import torch

GLL = "gll"      # SEM-NI: Gauss-Legendre-Lobatto, collocated with the nodes
GAUSS = "gauss"  # SEM: Legendre-Gauss


@dataclass(frozen=True)
class BoxSpec:
    """A structured hexahedral box of degree-p elements plus its physics.

    Geometry recipe (both sides implement it):
      * the Q_p node lattice of an axis-aligned box with `n` elements per axis,
        element edges `length / n`, nodes at the GLL points inside each element;
      * optional shear: every node (x, y, z) is moved to (x+d, y+d, z+d) with
        d = shear_amp * hx * sin(2*pi*(x - x0)/Lx), x the undeformed first
        coordinate and hx the element edge along x;
      * optional fiber a = (cos t, sin t, 0), t rising linearly from theta0 at
        z = z0 to theta1 at z = z0 + Lz (undeformed z), stored at every node;
      * optional sheet (with the fiber) s = (-sin t, cos t, 0) at every node, so
        that the cross-fiber direction is e_z.
    Physics: conductivity sigma = (sigma_l, sigma_t, sigma_n); with a fiber and
    a sheet the tensor is sigma_l a a^T + sigma_t s s^T + sigma_n n n^T; with a
    fiber and no sheet it is sigma_t*I + (sigma_l - sigma_t)*a a^T; without a
    fiber it is sigma_t*I.  `alpha` multiplies the mass matrix.
    """

    p: int
    n: tuple
    origin: tuple = (0.0, 0.0, 0.0)
    length: tuple = (1.0, 1.0, 1.0)
    shear_amp: float = 0.0
    fiber: bool = False
    theta0: float = 0.0
    theta1: float = 0.0
    sigma: tuple = (1.0, 1.0, 1.0)
    alpha: float = 1.0
    quad: str = GLL
    nq1d: int = 0  # 0 -> p+1
    sheet: bool = False

    @property
    def q(self) -> int:
        return self.nq1d if self.nq1d > 0 else self.p + 1

    @property
    def n_elem(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def n_dof(self) -> int:
        p = self.p
        return (p * self.n[0] + 1) * (p * self.n[1] + 1) * (p * self.n[2] + 1)

    def with_(self, **kw) -> "BoxSpec":
        return dataclasses.replace(self, **kw)


DEG = math.pi / 180.0

# Slab physics shared by the slab workloads: 20 x 7 x 3 mm, sigma in mS/mm,
# chi = 140 /mm, Cm = 0.01 uF/mm^2, dt = 0.05 ms -> alpha = chi*Cm/dt = 28.
SLAB_LEN = (20.0, 7.0, 3.0)
SLAB_SIGMA = (0.17, 0.019, 0.019)
SLAB_ALPHA = 140.0 * 0.01 / 0.05


def slab(p: int, n: tuple, quad: str = GLL, nq1d: int = 0) -> BoxSpec:
    """Sheared slab with fibers rotating -60..+60 degrees through the thickness."""
    return BoxSpec(p=p, n=tuple(n), length=SLAB_LEN, shear_amp=0.05, fiber=True,
                   theta0=-60 * DEG, theta1=60 * DEG, sigma=SLAB_SIGMA,
                   alpha=SLAB_ALPHA, quad=quad, nq1d=nq1d)


# Named workloads.
C1 = BoxSpec(p=2, n=(4, 4, 4))                             # unit cube, affine, sigma=1, alpha=1
C2 = slab(4, (40, 14, 6))                                  # 229,425 DOFs
C3_NI = slab(7, (128, 48, 24))                             # 51,086,841 DOFs, GLL q=8
C3_SEM = slab(7, (128, 48, 24), quad=GAUSS, nq1d=9)        # Gauss q=p+2
C4 = BoxSpec(p=4, n=(32, 32, 32), length=(16.0, 16.0, 16.0), fiber=True,
             theta0=-60 * DEG, theta1=60 * DEG, sigma=SLAB_SIGMA, alpha=SLAB_ALPHA)
C5 = BoxSpec(p=5, n=(128, 128, 64), length=(20.0, 20.0, 10.0), fiber=True,
             theta0=-60 * DEG, theta1=60 * DEG, sigma=SLAB_SIGMA, alpha=SLAB_ALPHA)

# The paper's slab mesh (Section 5.1: 76 x 24 x 12 hexahedra on the 20 x 7 x 3 mm
# slab, whose Q1..Q4 node counts are the DOF counts the paper tabulates), with
# the paper's orthotropic conductivities read as diffusivities (chi = Cm = 1)
# and alpha = 3 / (2 dt) for BDF2 at dt = 0.1 ms.  Fiber e_x, sheet e_y: the
# paper's fiber field is not available, so this stands in for the shapes only.
PAPER_SLAB_N = (76, 24, 12)
PAPER_SLAB_SIGMA = (0.07643, 0.03494, 0.01125)
PAPER_SLAB_ALPHA = 3.0 / (2.0 * 0.1)


def paper_slab(p: int, quad: str = GLL) -> BoxSpec:
    """The paper's slab mesh at degree p; SEM uses Legendre-Gauss with p+1 points."""
    return BoxSpec(p=p, n=PAPER_SLAB_N, length=SLAB_LEN, fiber=True, theta0=0.0, theta1=0.0,
                   sheet=True, sigma=PAPER_SLAB_SIGMA, alpha=PAPER_SLAB_ALPHA, quad=quad,
                   nq1d=p + 1 if quad == GAUSS else 0)


# The p-sweep: the same sheared slab at about 51M DOFs for every p
# (a 896 x 336 x 168 node lattice, rounded to whole elements).
SWEEP_ELEMS = {2: (448, 168, 84), 3: (299, 112, 56), 4: (224, 84, 42),
               5: (179, 67, 34), 6: (149, 56, 28), 7: (128, 48, 24)}


def sweep(p: int, quad: str = GLL, nq1d: int = 0) -> BoxSpec:
    return slab(p, SWEEP_ELEMS[p], quad=quad, nq1d=nq1d)


# Random draws ---------------------------------------------------------------

def generator(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def uniform(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """float64 U[lo, hi) of the given shape, reproducible from `seed`."""
    if isinstance(shape, int):
        shape = (shape,)
    t = torch.rand(tuple(shape), dtype=torch.float64, generator=generator(seed))
    return (t * (hi - lo) + lo).numpy()


def node_jitter(seed: int, n_dof: int, scale: float) -> np.ndarray:
    """Per-node displacement [n_dof][3], U[-scale, scale) in each component."""
    return uniform(seed, (n_dof, 3), -scale, scale)


def element_sigma(seed: int, batch: int, n_elem: int,
                  l_range=(0.1, 0.2), t_range=(0.01, 0.03)) -> np.ndarray:
    """Per-element conductivities [batch][n_elem][3] = (sigma_l, sigma_t, sigma_n),
    sigma_l ~ U[l_range], sigma_t ~ U[t_range], sigma_n = sigma_t."""
    s = np.empty((batch, n_elem, 3))
    s[..., 0] = uniform(seed, (batch, n_elem), *l_range)
    s[..., 1] = uniform(seed + 100003, (batch, n_elem), *t_range)
    s[..., 2] = s[..., 1]
    return s


# Aliev-Panfilov constants (dimensionless model of Aliev & Panfilov, 1996) and
# the scaling to physical units used by the full monodomain workload:
# V = v_rest + v_amp * u [mV], t = t_scale * tau [ms].  These are workload
# parameters handed to both sides as inputs.
AP_PARAMS = dict(k=8.0, a=0.15, eps0=0.002, mu1=0.2, mu2=0.3,
                 v_rest=-80.0, v_amp=100.0, t_scale=12.9)
# Membrane constants of the slab workloads: chi [1/mm], Cm [uF/mm^2].
CHI, CM = 140.0, 0.01
