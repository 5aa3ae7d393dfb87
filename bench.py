"""Benchmark of the matrix-free SEM / SEM-NI operator and its GMG-PCG solve on one GPU.

Default workload: the sheared slab 20 x 7 x 3 mm at about 51M DOFs and p = 4
(224 x 84 x 42 hexahedra, 51,243,525 DOFs), GLL quadrature (SEM-NI),
anisotropic rotating-fiber conductivity, alpha = chi*Cm/dt = 28; FP64 apply and
GMG-PCG with p-coarsening 4 -> 2 -> 1 and Chebyshev degree 3, random
right-hand side.  Every apply moves about 6 GB, far beyond the 256 MB Infinity
Cache, so the rates are HBM rates.

One timed step = one pass of the hot path on that input:
  * R back-to-back operator applies y = A x (FP64; --apply-reps, default 20 on
    meshes above 4M DOFs, else 100), then R launches of the kernel alone
    (y += A x) in FP64 and in FP32,
  * one FP64 GMG-PCG solve A u = f to ||r||/||f|| <= 1e-10 from u0 = 0,
  * one mixed-precision solve (FP32 V-cycle inside FP64 flexible CG), same tolerance.
`value` is the apply throughput in GDOF/s (unique mesh nodes per second) from
HIP events around the back-to-back applies inside the timed steps; the PCG
times are reported beside it.  Set-up (geometry, diagonals, eigenvalue
estimates) is outside the timed region, as in the paper.

After the timed steps, the same JSON line carries (default run, --no-sweep to skip):
  sweep      the metric over p = 2..7 on the ~51M-DOF slab: FP64 and FP32 kernel
             times, y = A x, PCG time-to-1e-10 FP64 vs mixed with iterations,
             each solve's byte model per iteration and its HBM fraction, and
             its true residual (b - A x recomputed with the library's apply;
             the GPU tests certify full-size solutions against the oracle);
  c3_gauss   the same for SEM (Gauss q = 9) at p = 7, 128 x 48 x 24 hexes;
  c2         the 229,425-DOF c2 slab (cache-resident, latency-bound).
`pcg_roofline` gives the main workload's solve against the HBM roofline: the
algorithmic bytes of every kernel of one PCG iteration (V-cycle applies,
smoother steps, transfer passes, CG vector kernels) divided by the measured
time per iteration.

Other workloads (--workload):
  slab-p{2..7}[-gauss]  the sheared slab refined to about 51M DOFs (p-sweep),
  c2                    sheared slab, 40 x 14 x 6 hexes at p = 4 (229,425 DOFs),
  c3 / c3-gauss         128 x 48 x 24 hexes at p = 7, SEM-NI / SEM (q = 9),
  c2-p{1..8}            the c2 slab at another degree (the matrix-based comparison
                        per degree),
  paper-slab-p{1..4}[-gauss]
                        the paper's 76 x 24 x 12 slab mesh (its tabulated DOF
                        counts) with orthotropic diffusivities and Chebyshev
                        degree 5, as in its solver set-up,
  c4                    32^3 box at p = 4 with a batch of 8 per-element
                        conductivity sets: the step's solve is a forward
                        GMG-PCG plus the adjoint gradient dL/dsigma,
  c5                    128 x 128 x 64 box at p = 5: the step's solve is one
                        IMEX monodomain time step (run --steps 100 for the
                        full 5 ms),
  c5-bdf2               the same with the paper's BDF2 partitioned scheme and
                        activation times.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def sem_reads_index(p, w):
    """Whether the Gauss (SEM) kernel reads the element-to-node index on these
    structured meshes: its lattice form (node numbers computed) runs in FP64 up
    to p = 6 and in FP32 at every degree (the library's choice, by measurement)."""
    return w == 8 and p > 6


def apply_kernel(spec):
    """The kernel that performs y += A x for this workload, its source file, and
    the model of the bytes one launch must move: one read of x, one read and one
    write of y, the 6 stored G entries per quadrature point and 1/det(sigma) per
    element (the mass weight W|J| is recovered from det G, so no W|J| is read),
    plus the element-to-node index where the Gauss kernel reads it (the lattice
    kernels compute node numbers)."""
    P = spec.p + 1
    base = "8*(x + y read + y write)*N + 48*n_elem*q^3 (G) + 8*n_elem (1/det sigma)"
    if spec.quad == "gll":
        return (f"ax_brick_kernel<double,{P}>", "ax_brick.hip", base)
    return (f"ax_sem_kernel<double,{P},{spec.q}>", "ax.hip",
            base + (" + 4*n_elem*(p+1)^3 (index)" if sem_reads_index(spec.p, 8) else ""))


def algorithmic_bytes(spec, n_elem, n_dof, w, quad):
    """Bytes one y += A x launch must move (see apply_kernel) in word size w."""
    q3 = spec.q ** 3
    P3 = (spec.p + 1) ** 3
    g = 6 * n_elem * q3 * w
    b = 3 * w * n_dof + g + w * n_elem
    if quad != "gll" and sem_reads_index(spec.p, w):
        b += 4 * n_elem * P3
    return b


def algorithmic_flops(spec, n_elem, n_dof, quad):
    P, q = spec.p + 1, spec.q
    if quad == "gll":
        return n_elem * (12 * P ** 4 + 15 * q ** 3) + 2 * n_dof
    return n_elem * (4 * (q * P ** 3 + q * q * P * P + q ** 3 * P) + 12 * q ** 4 + 17 * q ** 3)


def measured_traffic(kernel, source, workload):
    """HBM bytes per launch from the committed counter runs (profiles/counters.json:
    rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, each scaled by the same counter's
    reading for a copy of known size), and a label saying where they come from.
    The bytes are None when the kernel source changed since they were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_2205_05136_amd", "csrc", source)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    try:
        entry = json.load(open(os.path.join(ROOT, "profiles", "counters.json"))).get(
            f"{kernel}|{workload}")
    except (OSError, ValueError):
        entry = None
    if not entry:
        return None, "no counter run for this kernel and workload"
    if entry.get("source_sha") != sha:
        return None, (f"counters taken at kernel source sha {entry.get('source_sha')}, "
                      f"current {sha}: not reported")
    return (int(entry["read_bytes"] + entry["write_bytes"]),
            f"not measured in this run: profiles/counters.json, rocprofv3 --pmc FETCH_SIZE and "
            f"WRITE_SIZE (copy-calibrated) at {source} sha {sha}")


# p-multigrid degree sequences, measured on the 51M-DOF slab (PCG to 1e-10, FP64 and
# mixed, Chebyshev degree 3): halving the degree from p = 3, 5, 6, 7 costs 15-18
# iterations where these sequences need 9-12, and 20-23% of the solve time at p = 3, 5.
# On meshes of a few hundred thousand DOFs the solve is bound by launch latency and
# the extra levels cost more than the iterations they save (c2 slab at p = 3..7:
# 1.4-5.7 ms with halving against 2.0-7.0 ms), so small problems halve the degree.
QSEQ = {1: (), 2: (1,), 3: (2, 1), 4: (2, 1), 5: (3, 1), 6: (4, 2, 1), 7: (5, 3, 1)}
SMALL_DOFS = 4_000_000


def coarsening_for(p, n_dof=None):
    """p-coarsening chain from degree p down to 1: the measured sequences (above 7:
    steps of 2 until 7), or halving the degree for meshes under SMALL_DOFS."""
    seq = []
    if n_dof is not None and n_dof < SMALL_DOFS:
        while p > 1:
            p = max(1, p // 2)
            seq.append(p)
        return tuple(("p", q) for q in seq)
    while p > 7:
        p -= 2
        seq.append(p)
    seq += QSEQ[p]
    return tuple(("p", q) for q in seq)


def mg_plan(name, spec):
    """(coarsening chain, Chebyshev degree) of a workload's multigrid.  The
    paper-shaped slab follows the paper's set-up (degree 5) and, after the
    p-levels, coarsens the 76 x 24 x 12 mesh twice by octree (-> 19 x 6 x 3)."""
    if name.startswith("paper-slab"):
        return coarsening_for(spec.p, spec.n_dof) + (("h",), ("h",)), 5
    return coarsening_for(spec.p, spec.n_dof), 3


def parse_chain(text):
    """'p5,p3,p1,h' -> (("p", 5), ("p", 3), ("p", 1), ("h",))."""
    out = []
    for tok in text.split(","):
        tok = tok.strip()
        out.append(("h",) if tok == "h" else ("p", int(tok[1:])))
    return tuple(out)


def chain_str(p, chain):
    out, cur = [f"p{p}"], p
    for c in chain:
        out.append(f"p{c[1]}" if c[0] == "p" else f"h(p{cur})")
        cur = c[1] if c[0] == "p" else cur
    return " -> ".join(out)


def workload(name):
    import synth
    if name.startswith("paper-slab-p"):
        parts = name.split("-")
        p = int(parts[2][1:])
        gauss = len(parts) > 3 and parts[3] == "gauss"
        spec = synth.paper_slab(p, quad="gauss" if gauss else "gll")
        return spec, (f"the paper's slab mesh: 20x7x3 mm, 76x24x12 hexes, p={p}, "
                      f"{'SEM (Gauss q=p+1)' if gauss else 'SEM-NI (GLL)'}, orthotropic "
                      f"diffusivities {synth.PAPER_SLAB_SIGMA} mm^2/ms with fiber e_x and "
                      f"sheet e_y, alpha = 3/(2*0.1 ms)")
    if name == "c2":
        return synth.C2, "c2: sheared slab 20x7x3 mm, 40x14x6 hexes, p=4, SEM-NI (GLL), rotating fibers"
    if name.startswith("c2-p"):
        p = int(name[4:])
        spec = synth.slab(p, (40, 14, 6))
        return spec, f"the c2 slab (40x14x6 hexes) at p={p}, SEM-NI (GLL)"
    if name.startswith("slab-p"):
        parts = name.split("-")
        p = int(parts[1][1:])
        gauss = len(parts) > 2 and parts[2] == "gauss"
        spec = synth.sweep(p, quad="gauss" if gauss else "gll", nq1d=p + 2 if gauss else 0)
        return spec, (f"sheared slab at ~51M DOFs: {spec.n[0]}x{spec.n[1]}x{spec.n[2]} hexes, "
                      f"p={p}, {'SEM (Gauss q=p+2)' if gauss else 'SEM-NI (GLL)'}")
    if name == "c3":
        return synth.C3_NI, "c3: sheared slab 128x48x24 hexes, p=7, SEM-NI (GLL)"
    if name == "c3-gauss":
        return synth.C3_SEM, "c3: sheared slab 128x48x24 hexes, p=7, SEM (Gauss q=9)"
    if name == "c4":
        return synth.C4, ("c4: box 16 mm, 32^3 hexes, p=4, SEM-NI, 8 per-element conductivity "
                          "sets; forward GMG-PCG + adjoint gradient")
    if name == "c5":
        return synth.C5, ("c5: box 20x20x10 mm, 128x128x64 hexes, p=5, SEM-NI; IMEX monodomain "
                          "steps (Aliev-Panfilov + mixed-precision GMG-PCG)")
    if name == "c5-bdf2":
        return synth.C5, ("c5 with the paper's BDF2 partitioned scheme: box 20x20x10 mm, "
                          "128x128x64 hexes, p=5, SEM-NI; implicit gating, lumped ionic "
                          "current, activation times (Aliev-Panfilov + mixed-precision GMG-PCG)")
    raise SystemExit(f"unknown workload {name}")


def level_plan(spec, chain):
    """(p, elements per axis, points per axis, quadrature) of every multigrid
    level, finest first: p-steps lower the degree on the same elements, h-steps
    halve the elements; levels below the finest are GLL (SEM-NI)."""
    p, n = spec.p, tuple(spec.n)
    levels = [(p, n, spec.q, spec.quad)]
    for c in chain:
        if c[0] == "p":
            p = c[1]
        else:
            n = tuple(k // 2 for k in n)
        levels.append((p, n, p + 1, "gll"))
    return levels


def _nodes(p, n):
    return [p * k + 1 for k in n]


def apply_bytes(p, n, q, quad, w):
    """Algorithmic bytes of one y += A x launch on a level (apply_kernel's model)."""
    ne = n[0] * n[1] * n[2]
    N = math.prod(_nodes(p, n))
    b = 3 * w * N + 6 * w * ne * q ** 3 + w * ne
    return b + (4 * ne * (p + 1) ** 3 if quad != "gll" else 0)


def pcg_bytes_model(spec, chain, degree, coarse_degree, mixed):
    """Algorithmic bytes of the PCG solve, kernel by kernel, as the library
    launches them: one iteration is one V-cycle (word size 4 when mixed, else
    8), a dot product r.z (and r.z_old for the flexible CG of the mixed solve),
    p = z + beta p, q = A p in FP64, a dot product p.q, and the x, r update
    (which also clears q and, mixed, writes r in FP32).  Each V-cycle level
    above the coarsest runs `degree` smoother steps before and after the
    coarse correction (the first from zero, without a product; each other one
    an apply y += A x and a damped-Jacobi step reading x, b, A x and D^-1 and
    writing x and clearing A x), the residual apply, a three-pass restriction
    (b - A x read, intermediate lattices written and read, the coarse b
    written) and a three-pass prolongation (the last pass reads and writes x
    and clears A x); the coarsest level runs `coarse_degree` steps from zero.
    Levels below the finest clear their b on its last read.  Returns
    {"iteration": bytes, "initial": bytes, "parts": {kernel group: bytes}}."""
    w = 4 if mixed else 8
    lv = level_plan(spec, chain)
    parts = {}

    def add(k, b):
        parts[k] = parts.get(k, 0) + int(b)

    for l, (p, n, q, quad) in enumerate(lv):
        N = math.prod(_nodes(p, n))
        A = apply_bytes(p, n, q, quad, w)
        own_b = w * N if l > 0 else 0
        if l == len(lv) - 1:
            k = coarse_degree
            add("vcycle_apply", (k - 1) * A)
            add("vcycle_smoother", 3 * w * N + (k - 1) * 6 * w * N + own_b)
            continue
        k = degree
        add("vcycle_apply", 2 * k * A)
        add("vcycle_smoother", 3 * w * N + (2 * k - 1) * 6 * w * N + own_b)
        F = _nodes(p, n)
        C = _nodes(lv[l + 1][0], lv[l + 1][1])
        s1, s2, Nc = F[0] * C[1] * C[2], F[0] * F[1] * C[2], math.prod(C)
        add("restriction", w * (2 * N + 2 * s2 + 2 * s1 + Nc))
        add("prolongation", w * (Nc + 2 * s1 + 2 * s2 + 3 * N))
    N = spec.n_dof
    add("cg_apply_fp64", apply_bytes(spec.p, spec.n, spec.q, spec.quad, 8))
    add("cg_vectors", (8 + w + (w if mixed else 0)) * N   # r.z (and r.z_old)
        + (w + 16) * N                                    # p = z + beta p
        + 16 * N                                          # p.q
        + (56 + (4 if mixed else 0)) * N)                 # x, r update, q cleared
    initial = apply_bytes(spec.p, spec.n, spec.q, spec.quad, 8) + (32 + (4 if mixed else 0)) * N
    return {"iteration": sum(parts.values()), "initial": int(initial), "parts": parts}


def pcg_roofline(spec, chain, degree, ms, iters, mixed):
    """The solve against the HBM roofline: modelled bytes of the whole solve
    (initial residual + iterations) over its measured time."""
    m = pcg_bytes_model(spec, chain, degree, 2 * degree, mixed)
    total = m["initial"] + iters * m["iteration"]
    achieved = total / (ms * 1e-3) / 1e9
    return {"bytes_per_iteration": m["iteration"], "bytes_initial_residual": m["initial"],
            "bytes_per_iteration_by_kernel": m["parts"],
            "achieved_GBs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4)}


def _median(v):
    v = sorted(v)
    return v[len(v) // 2]


def cpu_baseline(spec, budget_s=12.0):
    """The oracle timed on the host cores, on bounded samples.

    value: the oracle's own apply on the benchmark's workload, row by row
    (dense element matrices of the elements around each DOF, as it stands,
    one thread), scaled to GDOF/s; the full matrix of a 51M-DOF mesh would
    not fit the host.  c2: the oracle's assembled CSR matrix of the c2 slab,
    its product timed with SciPy on one thread and with torch's sparse CSR
    on every host core (median of 5 runs each)."""
    import numpy as np
    import torch
    import synth
    from threadpoolctl import threadpool_limits
    from oracle import operator as oop
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    out = {}
    with threadpool_limits(1):
        x_fn = lambda g: np.sin(0.37 * np.asarray(g, dtype=np.float64))
        rng = np.random.default_rng(0)
        rows, t = 0, 0.0
        while t < budget_s:
            g = rng.integers(0, spec.n_dof, 16)
            t1 = time.perf_counter()
            oop.apply_rows(spec, x_fn, g)
            t += time.perf_counter() - t1
            rows += len(g)
    out.update({"value": rows / t / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
                "sample": (f"oracle row-by-row apply (dense element matrices of the elements "
                           f"around each DOF, one thread) on {rows} random rows of the "
                           f"benchmark's {spec.n_dof:,}-DOF mesh in {t:.1f} s, scaled to GDOF/s; "
                           f"the host has {ncpu} cores")})
    c2 = synth.C2
    with threadpool_limits(1):
        t0 = time.perf_counter()
        A, _, _ = oop.Problem(c2).assemble()
        t_asm = time.perf_counter() - t0
        x = synth.uniform(100, c2.n_dof)
        t1 = []
        for _ in range(5):
            a = time.perf_counter()
            A @ x
            t1.append(time.perf_counter() - a)
    nt = torch.get_num_threads()
    torch.set_num_threads(ncpu)
    try:
        At = torch.sparse_csr_tensor(torch.as_tensor(A.indptr, dtype=torch.int64),
                                     torch.as_tensor(A.indices, dtype=torch.int64),
                                     torch.as_tensor(A.data), size=A.shape)
        xt = torch.as_tensor(x)
        At @ xt
        tn = []
        for _ in range(5):
            a = time.perf_counter()
            At @ xt
            tn.append(time.perf_counter() - a)
    finally:
        torch.set_num_threads(nt)
    m1, mn = _median(t1), _median(tn)
    out["c2_csr_spmv"] = {
        "n_dof": c2.n_dof, "nnz": int(A.nnz),
        "scipy_1_thread": {"ms": round(m1 * 1e3, 3), "gdofs": round(c2.n_dof / m1 / 1e9, 5),
                           "cores": 1},
        "torch_csr_all_cores": {"ms": round(mn * 1e3, 3), "gdofs": round(c2.n_dof / mn / 1e9, 5),
                                "cores": ncpu},
        "assembly_s": round(t_asm, 1),
        "sample": "the oracle's assembled matrix of the c2 slab (Alg. 2's matrix-based path), "
                  "median of 5 products each; assembly excluded"}
    return out


def cpu_pcg_baseline(spec, chain, degree, max_dofs=1_000_000):
    """The oracle's GMG-PCG (explicit level matrices, prolongation matrices and
    V-cycle, the same chain and Chebyshev degrees, lambda_max by its own 10-step
    Lanczos) to 1e-10 from zero on the workload's right-hand side, timed on one
    host core.  Only for meshes the oracle assembles in seconds."""
    import synth
    from threadpoolctl import threadpool_limits
    from oracle import multigrid as omg
    from oracle import operator as oop
    from oracle import solvers as osol
    if spec.n_dof > max_dofs or spec.quad != "gll" or any(c[0] != "p" for c in chain):
        return None
    with threadpool_limits(1):
        t0 = time.perf_counter()
        mats, Ps, p = [oop.Problem(spec).assemble()[0]], [], spec.p
        for c in chain:
            mats.append(oop.Problem(spec, dof_p=c[1], quad="gll").assemble()[0])
            Ps.append(omg.prolongation_p(spec.n, p, c[1]))
            p = c[1]
        levels = []
        for A in mats:
            dinv = 1.0 / A.diagonal()
            levels.append((A, dinv, osol.lanczos_lambda_max(A, dinv, synth.uniform(7, A.shape[0]))))
        t_setup = time.perf_counter() - t0
        f = synth.uniform(2, spec.n_dof)
        t1 = time.perf_counter()
        x, it, rn = osol.cg(mats[0], f, rtol=1e-10,
                            M=lambda r: osol.vcycle(levels, Ps, r, degree, 2 * degree))
        t_solve = time.perf_counter() - t1
    return {"kind": "oracle", "cores": 1, "n_dof": spec.n_dof,
            "time_to_1e-10_ms": round(t_solve * 1e3, 1), "iterations": it,
            "setup_s": round(t_setup, 1),
            "sample": "oracle GMG-PCG with explicit SciPy level matrices (same chain, Chebyshev "
                      "degree, tolerance and right-hand side), one thread"}


def matrix_based(mf, op, x, t_mf_ms, spec, max_bytes=40e9):
    """The paper's matrix-based comparison on the GPU: assemble A in CSR
    (mfsem_csr_assemble) and time its product (mfsem_csr_spmv) beside the
    matrix-free kernel, outside the timed steps.  The top-level fields are the
    element pattern (every pair of nodes sharing an element, as a standard
    assembly stores it); `coupled` holds the same for the pattern without
    collocation's zeros.  Skipped when a matrix would exceed max_bytes."""
    if spec.quad != "gll":
        return {"skipped": "the assembled-matrix path covers GLL (SEM-NI) operators"}
    out = _csr_point(mf, op, x, t_mf_ms, spec, "element", max_bytes)
    out["coupled"] = _csr_point(mf, op, x, t_mf_ms, spec, "coupled", max_bytes)
    return out


def _csr_point(mf, op, x, t_mf_ms, spec, pattern, max_bytes):
    import ctypes
    import torch
    from paper_2205_05136_amd import _lib as L
    nnz = ctypes.c_int64()
    L.check(L.load().mfsem_csr_nnz(op.handle, mf.CsrMatrix.PATTERNS[pattern], ctypes.byref(nnz)))
    nbytes = 12 * nnz.value + 8 * (spec.n_dof + 1)
    if nbytes > max_bytes:
        return {"skipped": f"{nbytes / 1e9:.1f} GB matrix"}
    E = lambda: torch.cuda.Event(enable_timing=True)
    a, b = E(), E()
    a.record()
    A = mf.CsrMatrix(op, pattern)
    b.record()
    torch.cuda.synchronize()
    t_asm = a.elapsed_time(b)
    y = torch.empty_like(x)
    for _ in range(3):
        A.apply(x, out=y)
    R = 20
    a.record()
    for _ in range(R):
        A.apply(x, out=y)
    b.record()
    torch.cuda.synchronize()
    t_spmv = a.elapsed_time(b) / R
    moved = 12 * nnz.value + 8 * (spec.n_dof + 1) + 16 * spec.n_dof  # vals, cols, row_ptr, x, y
    out = {"nnz": nnz.value, "matrix_bytes": nbytes, "assemble_ms": round(t_asm, 3),
           "spmv_ms": round(t_spmv, 4), "spmv_gdofs": round(spec.n_dof / (t_spmv * 1e-3) / 1e9, 3),
           "spmv_hbm_frac": round(moved / (t_spmv * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "matrix_free_speedup": round(t_spmv / t_mf_ms, 2)}
    # the same matrix through the vendor sparse library (torch's CSR product on
    # the GPU, int32 indices), for comparison with the hand-written SpMV
    try:
        At = torch.sparse_csr_tensor(A.row_ptr.to(torch.int32), A.col, A.val,
                                     size=(spec.n_dof, spec.n_dof))
        yl = At @ x
        err = float(torch.linalg.norm(yl - y) / torch.linalg.norm(y))
        for _ in range(3):
            At @ x
        a.record()
        for _ in range(R):
            At @ x
        b.record()
        torch.cuda.synchronize()
        out["library_spmv_ms"] = round(a.elapsed_time(b) / R, 4)
        out["library_vs_own_rel_l2"] = err
        del At, yl
    except (RuntimeError, NotImplementedError) as exc:
        out["library_spmv_ms"] = None
        out["library_note"] = str(exc)[:200]
    del A
    torch.cuda.empty_cache()
    return out


def _timed(fn, reps):
    """Mean milliseconds per call of fn over `reps` back-to-back calls, from HIP
    events on the current stream (three untimed calls first)."""
    import torch
    for _ in range(3):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def measure_point(mf, spec, chain, degree, R, solves=3):
    """The metric at one configuration: FP64 and FP32 kernel times (y += A x,
    HIP events), y = A x through the binding, PCG to 1e-10 from zero in FP64 and
    mixed precision (median of `solves` after one untimed solve each), their
    iterations, true residuals, byte models and HBM fractions."""
    import torch
    import synth
    N = spec.n_dof
    t0 = time.perf_counter()
    ops, mg32 = mf.hierarchy(spec, coarsening=chain, degree=degree, precision=torch.float32)
    op = ops[0]
    mg64 = mf.Multigrid(ops, mg32.transfers, degree=degree, precision=torch.float64)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    g = torch.arange(N, device="cuda", dtype=torch.float64)
    x = torch.sin(0.37 * g)
    y = torch.zeros_like(x)
    x32, y32 = x.float(), torch.zeros(N, device="cuda", dtype=torch.float32)
    t_apply = _timed(lambda: op.apply(x, out=y), R)
    t_k64 = _timed(lambda: op.apply_add(x, y), R)
    t_k32 = _timed(lambda: op.apply_add(x32, y32), R)
    f = torch.as_tensor(synth.uniform(2, N), device="cuda")
    res = {}
    for tag, mg in (("fp64", mg64), ("mixed", mg32)):
        u, info = mf.pcg(op, f, mg=mg, rtol=1e-10, max_it=200)
        ts = []
        for _ in range(solves):
            torch.cuda.synchronize()
            a = time.perf_counter()
            u, info = mf.pcg(op, f, mg=mg, rtol=1e-10, max_it=200)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - a) * 1e3)
        ms = _median(ts)
        rr = float(torch.linalg.norm(f - op.apply(u)) / torch.linalg.norm(f))
        res[tag] = (u, ms, info.iters[0], rr)
    u64, u32 = res["fp64"][0], res["mixed"][0]
    kname, _, _ = apply_kernel(spec)
    b64 = algorithmic_bytes(spec, spec.n_elem, N, 8, spec.quad)
    b32 = algorithmic_bytes(spec, spec.n_elem, N, 4, spec.quad)
    out = {"n_dof": N, "n_elem": spec.n_elem, "elements": list(spec.n), "p": spec.p,
           "quadrature": spec.quad, "nq1d": spec.q, "multigrid": chain_str(spec.p, chain),
           "kernel": kname, "setup_s": round(setup, 2),
           "fp64_apply_ms": round(t_apply, 4), "fp64_apply_gdofs": round(N / t_apply / 1e6, 2),
           "fp64_kernel_ms": round(t_k64, 4), "fp64_kernel_gdofs": round(N / t_k64 / 1e6, 2),
           "fp64_kernel_hbm_frac": round(b64 / (t_k64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "fp32_kernel_ms": round(t_k32, 4), "fp32_kernel_gdofs": round(N / t_k32 / 1e6, 2),
           "fp32_kernel_hbm_frac": round(b32 / (t_k32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    for tag in ("fp64", "mixed"):
        _, ms, it, rr = res[tag]
        out[f"pcg_{tag}"] = {"ms": round(ms, 3), "iters": it, "ms_per_iteration": round(ms / it, 3),
                             "true_rel_residual": rr,
                             "roofline": pcg_roofline(spec, chain, degree, ms, it, tag == "mixed")}
    out["mixed_vs_fp64_rel_l2"] = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
    del ops, mg32, mg64, op, res, u64, u32, x, y, x32, y32, f
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slab-p4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the p = 2..7 sweep, c3 Gauss and c2 sections of the default run")
    ap.add_argument("--apply-reps", type=int, default=None,
                    help="applies per step (default 20 above 4M DOFs, else 100)")
    ap.add_argument("--coarsening", default=None,
                    help="multigrid chain below the finest level, e.g. p5,p3,p1 or p2,p1,h "
                         "(default: the workload's)")
    ap.add_argument("--cheb-degree", type=int, default=None,
                    help="Chebyshev degree of the smoother (default: the workload's)")
    ap.add_argument("--no-matrix-based", action="store_true",
                    help="skip the assembled-matrix (CSR) comparison")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run an elementwise copy of 2 x N doubles (HBM counter reference)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library has "
              f"no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2205_05136_amd as mf
    import synth

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    spec, desc = workload(args.workload)
    kind = {"c4": "grad", "c5": "monodomain", "c5-bdf2": "monodomain"}.get(args.workload, "pcg")
    if args.no_pcg and kind == "pcg":
        kind = None
    sweep = args.workload == "slab-p4" and not args.no_sweep and kind == "pcg"
    log(f"workload {args.workload}: {desc}; N = {spec.n_dof:,} DOFs, {spec.n_elem:,} elements")
    dev = "cuda"
    t0 = time.perf_counter()
    coarsening, cheb_degree = mg_plan(args.workload, spec)
    if args.coarsening:
        coarsening = parse_chain(args.coarsening)
    if args.cheb_degree:
        cheb_degree = args.cheb_degree
    B = 1
    if kind == "pcg":
        ops, mg32 = mf.hierarchy(spec, coarsening=coarsening, degree=cheb_degree,
                                 precision=torch.float32)
        op = ops[0]
        mg64 = mf.Multigrid(ops, mg32.transfers, degree=cheb_degree, precision=torch.float64)
        f = torch.as_tensor(synth.uniform(2, spec.n_dof), device=dev)
    elif kind == "grad":
        from paper_2205_05136_amd import autograd as ag
        B = 8
        sig = torch.as_tensor(synth.element_sigma(4, B, spec.n_elem), device=dev)
        fB = torch.as_tensor(synth.uniform(5, (B, spec.n_dof)), device=dev)
        ut = torch.as_tensor(synth.uniform(6, (B, spec.n_dof)), device=dev)
        solver = ag.Solver(spec, batch=B, coarsening=coarsening, degree=cheb_degree, rtol=1e-10,
                           precision=torch.float64)
        solver.set_sigma(sig)
        # the same forward and adjoint solves with the FP32 V-cycle (flexible FP64 CG)
        solver32 = ag.Solver(spec, batch=B, coarsening=coarsening, degree=cheb_degree,
                             rtol=1e-10, precision=torch.float32)
        solver32.set_sigma(sig)
        op = solver.ops[0]
        op32 = None
    elif kind == "monodomain":
        from paper_2205_05136_amd.monodomain import Monodomain, Stimulus
        sim = Monodomain(spec, dt=0.05, chi=synth.CHI, cm=synth.CM, ap_params=synth.AP_PARAMS,
                         stimulus=Stimulus((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 50.0, 2.0),
                         coarsening=coarsening, degree=cheb_degree, precision=torch.float32,
                         scheme="bdf2" if args.workload == "c5-bdf2" else "imex1")
        op = sim.op
    else:
        op = mf.Operator.from_spec(spec, store_f32=True)
    if kind == "grad":
        # the FP32 kernel is timed on the same mesh with the constant conductivity
        op32 = mf.Operator.from_spec(spec, store_f64=False, store_f32=True)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"set-up {t_setup:.2f} s")

    N = spec.n_dof
    x = torch.as_tensor(synth.uniform(100, B * N), device=dev)   # [batch][N], flattened
    y = torch.empty_like(x)
    x32 = torch.as_tensor(synth.uniform(100, N), device=dev).float()
    y32 = torch.empty_like(x32)
    opf = op if kind != "grad" else op32
    E = lambda: torch.cuda.Event(enable_timing=True)
    R = args.apply_reps or (20 if N > SMALL_DOFS else 100)

    def step(rec):
        ev = [E() for _ in range(10)]
        ev[0].record()
        for _ in range(R):
            op.apply(x, out=y)                 # full apply: clear y + operator kernel
        ev[1].record()
        y.zero_()
        ev[2].record()
        for _ in range(R):
            op.apply_add(x, y)                 # the operator kernel alone
        ev[3].record()
        y32.zero_()
        ev[4].record()
        for _ in range(R):
            opf.apply_add(x32, y32)            # FP32 operator kernel
        ev[5].record()
        if kind == "pcg":
            u64, i64 = mf.pcg(op, f, mg=mg64, rtol=1e-10, max_it=200)
            ev[6].record()
            u32, i32 = mf.pcg(op, f, mg=mg32, rtol=1e-10, max_it=200)
            ev[7].record()
            rec.setdefault("sol", (u64, u32))
            rec.setdefault("its", []).append((i64.iters[0], i32.iters[0]))
        elif kind == "grad":
            s = sig.clone().requires_grad_(True)
            u = ag.solve(s, fB, solver)
            ev[6].record()
            loss = 0.5 * ((u - ut) ** 2).sum()
            loss.backward()
            ev[7].record()
            rec.setdefault("grad", s.grad)
            s32 = sig.clone().requires_grad_(True)
            u32 = ag.solve(s32, fB, solver32)
            ev[8].record()
            (0.5 * ((u32 - ut) ** 2).sum()).backward()
            ev[9].record()
            rec.setdefault("grad32", s32.grad)
        elif kind == "monodomain":
            info = sim.step()
            ev[6].record()
            ev[7].record()
            rec.setdefault("its", []).append(info.iters[0])
        rec.setdefault("ev", []).append(ev)

    warm = {}
    for _ in range(args.warmup):
        step(warm)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} steps); timing {args.steps} steps")
    rec = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3
    log(f"timed steps done: {ms_step:.1f} ms per step")

    def mean_ms(a, b):
        return sum(ev[a].elapsed_time(ev[b]) for ev in rec["ev"]) / len(rec["ev"])

    t_apply = mean_ms(0, 1) / R
    t_kernel = mean_ms(2, 3) / R
    t_kernel32 = mean_ms(4, 5) / R
    NB = N * B
    gdofs = NB / (t_apply * 1e-3) / 1e9
    bytes64 = B * algorithmic_bytes(spec, spec.n_elem, N, 8, spec.quad)
    bytes32 = algorithmic_bytes(spec, spec.n_elem, N, 4, spec.quad)
    flops = B * algorithmic_flops(spec, spec.n_elem, N, spec.quad)
    achieved = bytes64 / (t_kernel * 1e-3) / 1e9
    kname, ksrc, kmodel = apply_kernel(spec)
    traffic, traffic_src = measured_traffic(kname, ksrc, args.workload)
    out = {
        "metric": "operator-apply GDOF/s and PCG time-to-1e-10, FP64 vs mixed, p=2..7",
        "value": round(gdofs, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_dof": N, "batch": B, "n_elem": spec.n_elem, "p": spec.p,
                   "quadrature": spec.quad, "nq1d": spec.q, "alpha": spec.alpha,
                   "sigma_mS_per_mm": list(spec.sigma),
                   "multigrid": chain_str(spec.p, coarsening)
                                + f", Chebyshev degree {cheb_degree} on [0.08, 1.2]*lambda_max"
                                + f" (10 CG steps), coarsest level Chebyshev degree {2 * cheb_degree}",
                   "parallelism": "single GPU"},
        "apply": {"reps_per_step": R, "fp64_ms": round(t_apply, 5), "fp64_kernel_ms": round(t_kernel, 5),
                  "fp64_kernel_gdofs": round(NB / (t_kernel * 1e-3) / 1e9, 3),
                  "fp32_kernel_ms": round(t_kernel32, 5),
                  "fp32_kernel_gdofs": round(N / (t_kernel32 * 1e-3) / 1e9, 3),
                  "fp32_hbm_frac": round(bytes32 / (t_kernel32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "fp64_tflops": round(flops / (t_kernel * 1e-3) / 1e12, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_source": traffic_src,
                     "kernel": kname,
                     "bytes_per_launch": int(bytes64),
                     "bytes_model": kmodel},
    }
    if kind == "pcg":
        t64 = mean_ms(5, 6)
        t32 = mean_ms(6, 7)
        u64, u32 = rec["sol"]
        r = f - op.apply(u64)
        rel_res = float(torch.linalg.norm(r) / torch.linalg.norm(f))
        r32 = f - op.apply(u32)
        rel_res32 = float(torch.linalg.norm(r32) / torch.linalg.norm(f))
        rel_mixed = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
        lam64 = mg64.lambdas()[:, 0].tolist()
        it64, it32 = rec["its"][0]
        out["pcg"] = {"fp64_ms": round(t64, 4), "mixed_ms": round(t32, 4),
                      "fp64_iters": it64, "mixed_iters": it32,
                      "fp64_ms_per_iteration": round(t64 / max(it64, 1), 4),
                      "mixed_ms_per_iteration": round(t32 / max(it32, 1), 4),
                      "fp64_true_rel_residual": rel_res, "mixed_true_rel_residual": rel_res32,
                      "mixed_vs_fp64_rel_l2": rel_mixed,
                      "lambda_max_per_level": [round(v, 5) for v in lam64],
                      "tol": 1e-10, "x0": "zero", "setup_s": round(t_setup, 3)}
        out["pcg_roofline"] = {
            "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "fp64": pcg_roofline(spec, coarsening, cheb_degree, t64, it64, False),
            "mixed": pcg_roofline(spec, coarsening, cheb_degree, t32, it32, True),
            "model": "algorithmic bytes of every kernel of the solve (pcg_bytes_model) / "
                     "measured solve time (HIP events)"}
    elif kind == "grad":
        g, g32 = rec["grad"], rec["grad32"]
        out["grad"] = {"batch": B, "forward_solve_ms": round(mean_ms(5, 6), 4),
                       "backward_ms": round(mean_ms(6, 7), 4),
                       "backward": "adjoint GMG-PCG (FP64, rtol 1e-10) + per-element dA/dsigma contraction",
                       "mixed_forward_solve_ms": round(mean_ms(7, 8), 4),
                       "mixed_backward_ms": round(mean_ms(8, 9), 4),
                       "mixed": "FP32 V-cycle inside flexible FP64 CG, same tolerance",
                       "mixed_vs_fp64_grad_rel_l2": float(torch.linalg.norm(g32 - g) / torch.linalg.norm(g)),
                       "grad_finite": bool(torch.isfinite(g).all()),
                       "setup_s": round(t_setup, 3)}
    elif kind == "monodomain":
        its = rec["its"]
        st = sim.stats
        k = len(its)
        out["monodomain"] = {"time_steps_timed": k, "dt_ms": 0.05,
                             "ms_per_time_step": round(mean_ms(5, 6), 4),
                             "ionic_rhs_ms": round(sum(st.ionic_ms[-k:]) / k, 4),
                             "solve_ms": round(sum(st.solve_ms[-k:]) / k, 4),
                             "pcg_iters_mean": round(sum(its) / k, 3),
                             "V_range_mV": [round(float(sim.V.min()), 3), round(float(sim.V.max()), 3)],
                             "sim_time_ms": round(sim.t, 4), "setup_s": round(t_setup, 3),
                             "scheme": sim.scheme}
        # every node has a largest |dV/dt| once a step has run; it marks an
        # activation only where the node depolarised, i.e. where that rate is an
        # upstroke's (above 10 mV/ms; resting tissue ahead of the front changes
        # orders of magnitude more slowly)
        up = (sim.act >= 0) & (sim.act_rate > 10.0)
        act = sim.act[up]
        out["monodomain"]["activated_fraction"] = round(act.numel() / sim.act.numel(), 5)
        out["monodomain"]["activation_ms_range"] = (
            [round(float(act.min()), 4), round(float(act.max()), 4)] if act.numel() else None)
        out["monodomain"]["max_rate_mV_per_ms"] = round(float(sim.act_rate.max()), 3)
        out["monodomain"]["activation"] = ("time of the largest |dV/dt| per node (step midpoint), "
                                           "counted where that rate exceeds 10 mV/ms")
    if kind == "pcg" and not args.no_matrix_based:
        out["matrix_based"] = matrix_based(mf, op, x, t_kernel, spec)
    if args.copy_ref:
        # y = x + 0: reads 8N and writes 8N bytes; its counter readings calibrate
        # the FETCH_SIZE / WRITE_SIZE of the operator kernel
        for _ in range(3):
            torch.add(x, 0.0, out=y)
        torch.cuda.synchronize()
        out["copy_ref_bytes"] = {"read": 8 * NB, "write": 8 * NB}
    if sweep:
        # free the main workload before the sweep builds its own hierarchies
        del ops, mg32, mg64, op, opf, rec, warm, x, y, x32, y32, f
        torch.cuda.empty_cache()
        out["sweep"] = {}
        for p in (2, 3, 4, 5, 6, 7):
            sp = synth.sweep(p)
            log(f"sweep p={p}: {sp.n_dof:,} DOFs ...")
            pt = measure_point(mf, sp, coarsening_for(p, sp.n_dof), 3, 20)
            out["sweep"][f"p{p}"] = pt
            log(f"  p={p}: FP64 kernel {pt['fp64_kernel_ms']} ms, PCG {pt['pcg_fp64']['ms']} / "
                f"{pt['pcg_mixed']['ms']} ms")
        sp = synth.C3_SEM
        log(f"c3 Gauss q=9: {sp.n_dof:,} DOFs ...")
        out["c3_gauss"] = measure_point(mf, sp, coarsening_for(7, sp.n_dof), 3, 20)
        out["c3_gauss"]["workload"] = workload("c3-gauss")[1]
        log("c2 ...")
        out["c2"] = measure_point(mf, synth.C2, coarsening_for(4, synth.C2.n_dof), 3, 100,
                                  solves=5)
        out["c2"]["workload"] = workload("c2")[1]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(spec)
        pcg_cpu = cpu_pcg_baseline(synth.C2, coarsening_for(4, synth.C2.n_dof), 3)
        if pcg_cpu is not None:
            out["cpu_baseline"]["c2_pcg"] = pcg_cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
