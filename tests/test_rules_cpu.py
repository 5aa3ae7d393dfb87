"""The compile-time 1D tables of the apply kernels (csrc/rules.hpp) against the
oracle's quadrature rules, weights and Lagrange matrices (Section 3: GLL nodes carry the
basis; SEM-NI integrates on them, SEM on Legendre-Gauss points).

The header is plain C++17, so it is compiled here with the host compiler and
its tables printed for every (P, Q) the kernels are instantiated for."""
import os
import subprocess

import numpy as np
import pytest

from oracle.basis import lagrange, lagrange_deriv
from oracle.quadrature import gauss, gll

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_05136_amd", "csrc")

# (P, Q) pairs of the SEM kernel (Q = P .. P + 2) and the SEM-NI P values
SEM_PQ = [(P, P + d) for P in range(2, 10) for d in range(3)]
GLL_P = list(range(2, 10))


def _program():
    lines = ["#include <cstdio>", '#include "rules.hpp"', "using namespace mfsem::rules;",
             "template <int N> void put(const char* tag, int P, int Q, const Vec<N>& a) {",
             "  std::printf(\"%s %d %d\", tag, P, Q);",
             "  for (int i = 0; i < N; ++i) std::printf(\" %.17g\", a.v[i]);",
             "  std::printf(\"\\n\");", "}", "int main() {"]
    for P in GLL_P:
        lines.append(f"  put(\"D\", {P}, {P}, GllTables<{P}>::D);")
    for P, Q in SEM_PQ:
        lines.append(f"  put(\"B\", {P}, {Q}, SemTables<{P}, {Q}>::B);")
        lines.append(f"  put(\"Dq\", {P}, {Q}, SemTables<{P}, {Q}>::Dq);")
        lines.append(f"  put(\"iw2\", {P}, {Q}, SemTables<{P}, {Q}>::iw2);")
    lines += ["  return 0;", "}"]
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module")
def tables(tmp_path_factory):
    d = tmp_path_factory.mktemp("rules")
    src, exe = d / "rules.cpp", d / "rules"
    src.write_text(_program())
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC,
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        tag, P, Q, *vals = line.split()
        got[(tag, int(P), int(Q))] = np.array([float(v) for v in vals])
    return got


def _close(a, b):
    # entries up to O(p^2); the two sides differ only in rounding
    return np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("P", GLL_P)
def test_gll_derivative_matrix(tables, P):
    x, _ = gll(P - 1)
    ref = lagrange_deriv(x, x)  # [c, m] = l_m'(x_c)
    assert _close(tables[("D", P, P)], ref.ravel())


@pytest.mark.parametrize("P,Q", SEM_PQ)
def test_sem_interpolation_and_collocation_derivative(tables, P, Q):
    xn, _ = gll(P - 1)
    xq, _ = gauss(Q)
    assert _close(tables[("B", P, Q)], lagrange(xn, xq).ravel())
    assert _close(tables[("Dq", P, Q)], lagrange_deriv(xq, xq).ravel())


@pytest.mark.parametrize("P,Q", SEM_PQ)
def test_sem_inverse_square_gauss_weights(tables, P, Q):
    _, w = gauss(Q)
    assert _close(tables[("iw2", P, Q)], 1.0 / w ** 2)
