"""The oracle's mesh steps (face-halo fill from neighbours, per-patch step sizes)
against the pins of tests/mesh_checks.py, and mutants of them that the pins
must catch."""
from __future__ import annotations

import os

import pytest

import oracle
from tests import mesh_checks as mc


def oracle_calls(lib=None):
    def fill(data, sizes, offsets, nb, dim, nq):
        return oracle.halo_fill(data, sizes, offsets, nb, dim, nq, lib=lib)

    def update_lts(data, sizes, offsets, dim, nq, dt, h):
        return oracle.batch_update_lts(data, sizes, offsets, dim, nq, dt, h, lib=lib)

    def update(data, sizes, offsets, nb, dim, nq, dt, h):
        return update_lts(fill(data, sizes, offsets, nb, dim, nq), sizes, offsets, dim, nq, dt, h)

    def local_dt(lam, h, dim, cfl):
        return oracle.local_dt(lam, h, dim, cfl, lib=lib)

    return fill, update, update_lts, local_dt


MESHES = [(3, 4, 2, True), (3, 4, 2, False), (4, 3, 2, True), (2, 5, 2, False), (2, 3, 3, True), (2, 3, 3, False),
          (3, 2, 3, True)]


@pytest.mark.parametrize("n,p,dim,periodic", MESHES)
def test_mesh_step_equals_big_patch(n, p, dim, periodic):
    _, update, _, _ = oracle_calls()
    mc.check_big_patch_equivalence(update, n, p, dim, periodic)


@pytest.mark.parametrize("n,p,dim,periodic", [(3, 4, 2, True), (4, 2, 2, False), (2, 3, 3, False), (3, 2, 3, True)])
def test_fill_writes_face_halos_only(n, p, dim, periodic):
    fill, _, _, _ = oracle_calls()
    mc.check_fill_leaves_the_rest(fill, n, p, dim, periodic)


@pytest.mark.parametrize("p,dim", [(5, 2), (3, 3)])
def test_per_patch_step_sizes(p, dim):
    _, _, update_lts, _ = oracle_calls()
    mc.check_per_patch_step_sizes(update_lts, p, dim)


def test_local_step_sizes():
    _, _, _, local_dt = oracle_calls()
    mc.check_local_dt(local_dt)


def test_peano_order_is_a_continuous_curve():
    from paper_2306_16731_amd import workloads as wl
    for n in (3, 9, 27):
        cells = wl.mesh_order(n, 2)
        assert len(set(cells)) == n * n
        assert all(abs(a[0] - b[0]) + abs(a[1] - b[1]) == 1 for a, b in zip(cells, cells[1:]))


def test_neighbor_tables_are_symmetric():
    from paper_2306_16731_amd import workloads as wl
    for n, dim, periodic in ((9, 2, True), (4, 2, False), (4, 3, True), (3, 3, False)):
        m = wl.make_mesh(n, 2, dim=dim, periodic=periodic)
        for t in range(m.batch.num_patches):
            for a in range(dim):
                for s in (0, 1):
                    nb = m.neighbors[t, 2 * a + s]
                    if nb >= 0:
                        assert m.neighbors[nb, 2 * a + (1 - s)] == t
                    else:
                        assert not periodic and m.coords[t][a] == (0 if s == 0 else n - 1)


MUTANTS = [
    ("fill reads the second layer", "g[n] = (s == 0) ? p : 1;", "g[n] = (s == 0) ? p - 1 : 1;"),
    ("fill reads the far side of the neighbour", "g[n] = (s == 0) ? p : 1;", "g[n] = (s == 0) ? 1 : p;"),
    ("fill writes the opposite halo", "h[n] = (s == 0) ? 0 : p + 1;", "h[n] = (s == 0) ? p + 1 : 0;"),
    ("per-patch update uses patch 0's dt", "dt[t], h[t], gamma);", "dt[0], h[t], gamma);"),
    ("per-patch update uses patch 0's h", "dt[t], h[t], gamma);", "dt[t], h[0], gamma);"),
    ("local step size without the dimension", "cfl * h[t] / (dim * lambda[t])", "cfl * h[t] / lambda[t]"),
    ("local step size of the first patch", "cfl * h[t] / (dim * lambda[t])", "cfl * h[t] / (dim * lambda[0])"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mesh_mutant_is_caught(name, old, new, tmp_path):
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1, f"mutation site not unique / missing: {old!r}"
    path = os.path.join(tmp_path, "mutant.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = oracle.load(oracle.build(path, os.path.join(tmp_path, "libmutant.so")))
    fill, update, update_lts, local_dt = oracle_calls(lib)
    checks = [
        ("fill", lambda: mc.check_fill_leaves_the_rest(fill, 3, 4, 2, False)),
        ("big patch 2D", lambda: mc.check_big_patch_equivalence(update, 3, 4, 2, True)),
        ("big patch 3D", lambda: mc.check_big_patch_equivalence(update, 2, 3, 3, False)),
        ("per-patch dt", lambda: mc.check_per_patch_step_sizes(update_lts, 5, 2)),
        ("local dt", lambda: mc.check_local_dt(local_dt)),
    ]
    for check_name, check in checks:
        try:
            check()
        except (AssertionError, ValueError):
            print(f"mutant '{name}' caught by: {check_name}")
            return
    pytest.fail(f"mutant '{name}' passes every pin")
