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
