"""Helpers shared by the GPU parity tests (oracle on the CPU, HIP path through
the C ABI on cuda:0)."""
import functools
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import multigrid as omg
from oracle import operator as oop
from oracle import solvers as osol

DEV = "cuda"


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def to_np(t):
    return t.detach().double().cpu().numpy()


@functools.lru_cache(maxsize=32)
def oracle_problem(spec, dof_p=None, sigma_seed=None, jitter=None):
    sigma = None
    if sigma_seed is not None:
        sigma = synth.element_sigma(sigma_seed, 1, spec.n_elem)[0]
    jit = None
    if jitter is not None:
        seed, scale = jitter
        jit = synth.node_jitter(seed, spec.n_dof, scale)
    prob = oop.Problem(spec, dof_p=dof_p, sigma=sigma, jitter=jit)
    A, M, K = prob.assemble()
    return prob, A, M, K


def jitter_scale(spec):
    h = min(spec.length[i] / spec.n[i] for i in range(3))
    return 0.02 * h / spec.p
