"""Benchmark of the matrix-free SEM-NI operator and its GMG-PCG solve on one GPU.

Default workload: the sheared slab 20 x 7 x 3 mm with 40 x 14 x 6 hexahedra at
p = 4, GLL quadrature (SEM-NI), anisotropic rotating-fiber conductivity,
alpha = chi*Cm/dt = 28 (229,425 DOFs); FP64 apply and GMG-PCG with
p-coarsening 4 -> 2 -> 1 and Chebyshev degree 3, random right-hand side.

One timed step = one pass of the hot path on that input:
  * R back-to-back operator applies y = A x (FP64; --apply-reps, default 100),
    then R launches of the kernel alone (y += A x) in FP64 and in FP32,
  * one FP64 GMG-PCG solve A u = f to ||r||/||f|| <= 1e-10 from u0 = 0,
  * one mixed-precision solve (FP32 V-cycle inside FP64 flexible CG), same tolerance.
`value` is the apply throughput in GDOF/s (unique mesh nodes per second) from
HIP events around the back-to-back applies inside the timed steps; the PCG
times are reported beside it.  Set-up (geometry, diagonals, eigenvalue
estimates) is outside the timed region, as in the paper.

Other workloads (--workload):
  slab-p{2..7}[-gauss]  the sheared slab refined to about 51M DOFs (p-sweep),
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


def apply_kernel(spec):
    """The kernel that performs y += A x for this workload, its source file, and
    the model of the bytes one launch must move: one read of x, one read and one
    write of y, the 6 stored G entries per quadrature point and 1/det(sigma) per
    element (the mass weight W|J| is recovered from det G, so no W|J| is read),
    plus the element-to-node index for the Gauss kernel (the lattice kernel
    computes node numbers)."""
    P = spec.p + 1
    if spec.quad == "gll":
        return (f"ax_brick_kernel<double,{P}>", "ax_brick.hip",
                "8*(x + y read + y write)*N + 48*n_elem*q^3 (G) + 8*n_elem (1/det sigma)")
    return (f"ax_sem_kernel<double,{P},{spec.q}>", "ax.hip",
            "8*(x + y read + y write)*N + 48*n_elem*q^3 (G) + 8*n_elem (1/det sigma) "
            "+ 4*n_elem*(p+1)^3 (index)")


def algorithmic_bytes(spec, n_elem, n_dof, w, quad):
    """Bytes one y += A x launch must move (see apply_kernel) in word size w."""
    q3 = spec.q ** 3
    P3 = (spec.p + 1) ** 3
    g = 6 * n_elem * q3 * w
    if quad == "gll":
        return 3 * w * n_dof + g + w * n_elem
    return 3 * w * n_dof + g + w * n_elem + 4 * n_elem * P3


def algorithmic_flops(spec, n_elem, n_dof, quad):
    P, q = spec.p + 1, spec.q
    if quad == "gll":
        return n_elem * (12 * P ** 4 + 15 * q ** 3) + 2 * n_dof
    return n_elem * (4 * (q * P ** 3 + q * q * P * P + q ** 3 * P) + 12 * q ** 4 + 17 * q ** 3)


def measured_traffic(kernel, source, workload):
    """HBM bytes per launch from the committed counter runs (profiles/counters.json),
    or None when the kernel source changed since they were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_2205_05136_amd", "csrc", source)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    try:
        entry = json.load(open(os.path.join(ROOT, "profiles", "counters.json"))).get(
            f"{kernel}|{workload}")
    except (OSError, ValueError):
        return None
    if not entry or entry.get("source_sha") != sha:
        return None
    return int(entry["read_bytes"] + entry["write_bytes"])


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


def cpu_baseline(spec, budget_s=20.0):
    """The oracle's matrix-based apply (assembled CSR SpMV, SciPy, one thread)
    on the same mesh, timed on the host cores."""
    import numpy as np
    import synth
    from oracle import operator as oop
    if spec.n_elem > 4000:
        # too large to assemble: rows of A x one by one from the element matrices
        x_fn = lambda g: np.sin(0.37 * np.asarray(g, dtype=np.float64))
        rng = np.random.default_rng(0)
        rows, t = 0, 0.0
        while t < budget_s:
            g = rng.integers(0, spec.n_dof, 16)
            t1 = time.perf_counter()
            oop.apply_rows(spec, x_fn, g)
            t += time.perf_counter() - t1
            rows += len(g)
        return {"value": rows / t / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
                "sample": (f"oracle row-by-row apply (dense element matrices of the elements "
                           f"around each DOF) on {rows} random rows of the full mesh in {t:.1f} s; "
                           f"assembling the full matrix at {spec.n_elem:,} elements is beyond "
                           f"this baseline's time budget")}
    t0 = time.perf_counter()
    prob = oop.Problem(spec)
    A, _, _ = prob.assemble()
    t_asm = time.perf_counter() - t0
    x = synth.uniform(100, prob.n_dof)
    reps, t_spmv = 0, 0.0
    while t_spmv < budget_s and reps < 200:
        t1 = time.perf_counter()
        A @ x
        t_spmv += time.perf_counter() - t1
        reps += 1
    per = t_spmv / reps
    return {"value": prob.n_dof / per / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle assembled-CSR SpMV (SciPy, single thread) on the full workload "
                       f"mesh, {reps} applies in {t_spmv:.1f} s ({per * 1e3:.2f} ms each); "
                       f"element-matrix assembly {t_asm:.1f} s excluded; host has "
                       f"{os.cpu_count()} logical CPUs")}


def cpu_pcg_baseline(spec, chain, degree, max_dofs=1_000_000):
    """The oracle's GMG-PCG (explicit level matrices, prolongation matrices and
    V-cycle, the same chain and Chebyshev degrees, lambda_max by its own 10-step
    Lanczos) to 1e-10 from zero on the workload's right-hand side, timed on the
    host beside the GPU solve.  Only for meshes the oracle assembles in seconds."""
    import numpy as np
    import synth
    from oracle import multigrid as omg
    from oracle import operator as oop
    from oracle import solvers as osol
    if spec.n_dof > max_dofs or spec.quad != "gll" or any(c[0] != "p" for c in chain):
        return None
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
    return {"kind": "oracle", "cores": 1, "time_to_1e-10_ms": round(t_solve * 1e3, 1),
            "iterations": it, "setup_s": round(t_setup, 1),
            "sample": "oracle GMG-PCG with explicit SciPy level matrices (same chain, Chebyshev "
                      "degree, tolerance and right-hand side), one thread"}


def matrix_based(mf, op, x, t_mf_ms, spec, max_bytes=40e9):
    """The paper's matrix-based comparison on the GPU: assemble A in CSR
    (mfsem_csr_assemble) and time its product (mfsem_csr_spmv) beside the
    matrix-free kernel, outside the timed steps.  Skipped when the matrix would
    exceed max_bytes."""
    import ctypes
    import torch
    from paper_2205_05136_amd import _lib as L
    if spec.quad != "gll":
        return {"skipped": "the assembled-matrix path covers GLL (SEM-NI) operators"}
    nnz = ctypes.c_int64()
    L.check(L.load().mfsem_csr_nnz(op.handle, ctypes.byref(nnz)))
    nbytes = 12 * nnz.value + 8 * (spec.n_dof + 1)
    if nbytes > max_bytes:
        return {"skipped": f"{nbytes / 1e9:.1f} GB matrix"}
    E = lambda: torch.cuda.Event(enable_timing=True)
    a, b = E(), E()
    a.record()
    A = mf.CsrMatrix(op)
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
    del A
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=100)
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
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has "
              f"no multi-GPU path in this build", file=sys.stderr)
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
    log(f"workload {args.workload}: {desc}; N = {spec.n_dof:,} DOFs, {spec.n_elem:,} elements")
    dev = "cuda"
    t0 = time.perf_counter()
    coarsening, cheb_degree = mg_plan(args.workload, spec)
    if args.coarsening:
        coarsening = parse_chain(args.coarsening)
    if args.cheb_degree:
        cheb_degree = args.cheb_degree
    B = 1
    extra = None
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
    R = args.apply_reps

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
    rec = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3

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
                     "traffic": measured_traffic(kname, ksrc, args.workload),
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
        if sim.scheme == "bdf2":
            act = sim.act[sim.act >= 0]
            out["monodomain"]["activated_fraction"] = round(act.numel() / sim.act.numel(), 5)
            out["monodomain"]["activation_ms_range"] = (
                [round(float(act.min()), 4), round(float(act.max()), 4)] if act.numel() else None)
    if kind == "pcg" and not args.no_matrix_based:
        out["matrix_based"] = matrix_based(mf, op, x, t_kernel, spec)
    if args.copy_ref:
        # y = x + 0: reads 8N and writes 8N bytes; its counter readings calibrate
        # the FETCH_SIZE / WRITE_SIZE of the operator kernel
        for _ in range(3):
            torch.add(x, 0.0, out=y)
        torch.cuda.synchronize()
        out["copy_ref_bytes"] = {"read": 8 * NB, "write": 8 * NB}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(spec)
        if kind == "pcg":
            pcg_cpu = cpu_pcg_baseline(spec, coarsening, cheb_degree)
            if pcg_cpu is not None:
                out["cpu_baseline"]["pcg"] = pcg_cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
