"""The pins can tell a wrong oracle from a right one.

Each case below plants one plausible mistake into a copy of the oracle's C
source (on the CPU, in a temporary directory), builds it, and requires that at
least one pin from ``tests/invariants.py`` fails on it.  A mutant that passes
every pin would mean the pins leave that part of the oracle unchecked.
"""
from __future__ import annotations

import os
import tempfile

import pytest

import oracle
from tests import invariants as inv

# (name, original text, planted text)
MUTANTS = [
    ("dissipation factor 1 instead of 1/2", "fhat[q] = 0.5 * (fL[q] + fR[q]) - 0.5 * s",
     "fhat[q] = 0.5 * (fL[q] + fR[q]) - 1.0 * s"),
    ("anti-dissipation", "fhat[q] = 0.5 * (fL[q] + fR[q]) - 0.5 * s", "fhat[q] = 0.5 * (fL[q] + fR[q]) + 0.5 * s"),
    ("dissipation dropped", "fhat[q] = 0.5 * (fL[q] + fR[q]) - 0.5 * s", "fhat[q] = 0.5 * (fL[q] + fR[q]) - 0.0 * s"),
    ("central average dropped", "fhat[q] = 0.5 * (fL[q] + fR[q])", "fhat[q] = fL[q]"),
    ("update sign flipped", "double d = fleft[q] - fright[q];", "double d = fright[q] - fleft[q];"),
    ("update scaled by dt*h", "double r = dt / h;", "double r = dt * h;"),
    ("pressure missing in momentum flux", "if (a == n) v = v + p;", "if (a == n) v = v;"),
    ("pressure on every momentum", "if (a == n) v = v + p;", "v = v + p;"),
    ("pressure missing in energy flux", "(q[nq - 1] + p) * un", "q[nq - 1] * un"),
    ("signed instead of absolute velocity", "fabs(un) + c", "un + c"),
    ("sound speed missing", "fabs(un) + c", "fabs(un) + 0.0 * c"),
    ("velocity of axis x everywhere", "double un = q[1 + n] / rho;", "double un = q[1] / rho;"),
    ("mass flux of axis x everywhere", "f[0] = q[1 + n];", "f[0] = q[1];"),
    ("gamma instead of gamma - 1", "(gamma - 1.0) * (E", "gamma * (E"),
    ("kinetic energy without 1/2", "(E - 0.5 * m2 / rho)", "(E - m2 / rho)"),
    ("kinetic energy ignores the last momentum", "for (int a = 0; a < ora_nmom(nq); ++a) m2", "for (int a = 0; a < 2; ++a) m2"),
    ("sound speed without gamma", "sqrt(gamma * p / rho)", "sqrt(p / rho)"),
    ("x and y swapped in the layout", "((kk * w + (size_t)j) * w + (size_t)i)", "((kk * w + (size_t)i) * w + (size_t)j)"),
    ("only the last axis enters the update", "D[q] = (n == 0) ? d : D[q] + d;", "D[q] = d;"),
    ("eigenvalue reduction skips the last axis", "for (int n = 0; n < dim; ++n) {\n                    double f[ORA_MAXQ], lam;",
     "for (int n = 0; n < dim - 1; ++n) {\n                    double f[ORA_MAXQ], lam;"),
    ("eigenvalue of the minimum", "return (a > b) ? a : b;", "return (a < b) ? a : b;"),
    ("max that drops NaN", "    if (a != a) return a;\n    if (b != b) return b;\n", ""),
    ("periodic halo 0 takes interior 1", "P + ora_vol(p, dim, 0, j, k, nq), P + ora_vol(p, dim, p, j, k, nq)",
     "P + ora_vol(p, dim, 0, j, k, nq), P + ora_vol(p, dim, 1, j, k, nq)"),
    ("right face uses the left neighbour", "ora_rusanov(qc, qh, n, nq, gamma, fright);", "ora_rusanov(qc, ql, n, nq, gamma, fright);"),
    ("corner volume read", "lo[n] -= 1;", "lo[n] -= 1; if (n == 1) lo[0] -= (i == 1);"),
]


def _checks(step):
    """Pins, cheapest first.  Each returns normally when the pin holds."""
    return [
        ("constant 2D", lambda: inv.check_constant_state(step, 2, 5)),
        ("constant 3D", lambda: inv.check_constant_state(step, 3, 5)),
        ("conservation 2D", lambda: inv.check_conservation(step, 2, 5)),
        ("conservation 3D", lambda: inv.check_conservation(step, 3, 5)),
        ("mirror 2D", lambda: inv.check_mirror(step, 2, 5)),
        ("mirror 3D", lambda: inv.check_mirror(step, 3, 5)),
        ("permutation 2D", lambda: inv.check_permutation(step, 2, 5)),
        ("permutation 3D", lambda: inv.check_permutation(step, 3, 5)),
        ("dimension reduction", lambda: inv.check_dimension_reduction(step)),
        ("passive scalar", lambda: inv.check_passive_scalar(step)),
        ("corners", lambda: inv.check_corner_independence(step, 2, 5)),
        ("nan", lambda: inv.check_nan_propagates(step, 2, 5)),
        ("acoustic 2D", lambda: inv.check_acoustic_convergence(step, 2, 5, (1, 1), sizes=(16, 32, 64))),
        ("acoustic 3D", lambda: inv.check_acoustic_convergence(step, 3, 5, (0, 0, 1), sizes=(16, 32, 64))),
    ]


@pytest.mark.slow
def test_unmutated_source_passes_every_pin():
    lib = oracle.load()

    def step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic):
        return oracle.batch_update(data, sizes, offsets, dim, nq, dt, h, gamma, periodic, lib=lib)

    for name, check in _checks(step):
        check()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1, f"mutation site not unique / missing: {old!r}"
    path = os.path.join(tmp_path, "mutant.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = oracle.load(oracle.build(path, os.path.join(tmp_path, "libmutant.so")))

    def step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic):
        return oracle.batch_update(data, sizes, offsets, dim, nq, dt, h, gamma, periodic, lib=lib)

    for check_name, check in _checks(step):
        try:
            check()
        except (AssertionError, FloatingPointError, ValueError):
            print(f"mutant '{name}' caught by: {check_name}")
            return
    pytest.fail(f"mutant '{name}' passes every pin")
