"""Host logic of the benchmark: multigrid chains, workloads and the byte model
(CPU only; no GPU and no oracle)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
import synth  # noqa: E402


def test_parse_and_print_chains():
    c = bench.parse_chain("p5, p3,p1,h")
    assert c == (("p", 5), ("p", 3), ("p", 1), ("h",))
    assert bench.chain_str(7, c) == "p7 -> p5 -> p3 -> p1 -> h(p1)"


@pytest.mark.parametrize("p", range(1, 12))
def test_coarsening_reaches_degree_one(p):
    for n_dof in (None, 10 ** 5, 10 ** 8):
        seq = [q for _, q in bench.coarsening_for(p, n_dof)]
        assert all(a > b for a, b in zip([p] + seq, seq))   # strictly decreasing
        assert (seq[-1] if seq else p) == 1


def test_measured_sequences_on_large_meshes_and_halving_on_small():
    big = 51_086_841
    assert bench.coarsening_for(4, big) == (("p", 2), ("p", 1))       # the c2 chain
    assert bench.coarsening_for(7, big) == (("p", 5), ("p", 3), ("p", 1))
    assert bench.coarsening_for(3, big) == (("p", 2), ("p", 1))
    assert bench.coarsening_for(7, 100_000) == (("p", 3), ("p", 1))
    assert bench.coarsening_for(5, 100_000) == (("p", 2), ("p", 1))


def test_workloads_and_plans():
    for name in ("c2", "c2-p3", "slab-p4", "slab-p7-gauss", "c3", "c3-gauss", "c4", "c5",
                 "c5-bdf2", "paper-slab-p1", "paper-slab-p4-gauss"):
        spec, desc = bench.workload(name)
        chain, deg = bench.mg_plan(name, spec)
        assert desc and deg in (3, 5)
        if name.startswith("paper-slab"):
            assert chain[-2:] == (("h",), ("h",)) and deg == 5
            assert spec.n == synth.PAPER_SLAB_N and spec.sheet
    assert bench.mg_plan("c2", synth.C2)[0] == (("p", 2), ("p", 1))
    with pytest.raises(SystemExit):
        bench.workload("no-such-workload")


def test_byte_model_at_p4():
    """117 B/DOF at p = 4 on the 51M-DOF slab (x, y read, y write, G, 1/det sigma)."""
    spec = synth.sweep(4)
    b = bench.algorithmic_bytes(spec, spec.n_elem, spec.n_dof, 8, "gll")
    assert b == 24 * spec.n_dof + 48 * spec.n_elem * 125 + 8 * spec.n_elem
    assert 116 < b / spec.n_dof < 118


def test_pcg_byte_model_counts_every_kernel():
    """The solve's byte model at p = 4 (chain 4 -> 2 -> 1, Chebyshev degree 3,
    coarsest degree 6): the V-cycle runs 2k applies on each level above the
    coarsest and coarse_degree - 1 on the coarsest, 2k smoother steps per level
    (one from zero), and the CG adds one FP64 apply and 112 B/DOF of vector
    traffic (r.z 16, p update 24, p.q 16, x/r update 56); the mixed V-cycle
    moves half the V-cycle bytes."""
    spec = synth.sweep(4)
    chain = bench.coarsening_for(4, spec.n_dof)
    m64 = bench.pcg_bytes_model(spec, chain, 3, 6, False)
    m32 = bench.pcg_bytes_model(spec, chain, 3, 6, True)
    A = [bench.apply_bytes(p, spec.n, p + 1, "gll", 8) for p in (4, 2, 1)]
    assert m64["parts"]["vcycle_apply"] == 6 * A[0] + 6 * A[1] + 5 * A[2]
    assert m64["parts"]["cg_apply_fp64"] == bench.algorithmic_bytes(spec, spec.n_elem,
                                                                    spec.n_dof, 8, "gll")
    assert m64["parts"]["cg_vectors"] == 112 * spec.n_dof
    N = [bench.math.prod(bench._nodes(p, spec.n)) for p in (4, 2, 1)]
    # per level: 3 words from zero + 5 steps of 6 words, + 1 word clearing b below the finest
    assert m64["parts"]["vcycle_smoother"] == 8 * (33 * N[0] + 34 * N[1] + (3 + 5 * 6 + 1) * N[2])
    for k in ("vcycle_apply", "vcycle_smoother", "restriction", "prolongation"):
        assert 2 * m32["parts"][k] == m64["parts"][k]
    assert m64["iteration"] == sum(m64["parts"].values())
    # about 75 GB per FP64 iteration on the 51M-DOF slab
    assert 70e9 < m64["iteration"] < 80e9 and 40e9 < m32["iteration"] < 47e9


def test_level_plan_follows_the_chain():
    spec = synth.paper_slab(4)
    lv = bench.level_plan(spec, (("p", 2), ("p", 1), ("h",), ("h",)))
    assert [l[0] for l in lv] == [4, 2, 1, 1, 1]
    assert lv[-1][1] == (19, 6, 3) and all(l[3] == "gll" for l in lv)
    g = bench.level_plan(synth.C3_SEM, (("p", 5),))
    assert g[0][2:] == (9, "gauss") and g[1][2:] == (6, "gll")
