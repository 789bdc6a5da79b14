"""Pins of the mesh steps around the kernel: face-halo fill from neighbouring
patches, per-patch (local) step sizes, and the update with per-patch dt and h.

Each check takes the implementation under test as callables, so the same pins
hold the CPU oracle (tests/test_oracle_mesh.py) and the HIP path
(tests/test_gpu_mesh.py):

    fill(data, sizes, offsets, neighbors, dim, nq) -> new array with the face halos filled
    update(data, sizes, offsets, neighbors, dim, nq, dt[T], h[T]) -> (out, lambda)
        one step with face halos taken from the neighbours (fill + per-patch update)
    local_dt(lam, h, dim, cfl) -> dt[T]

The reference of the mesh checks is not the code under test: a periodic (or
bounded) domain tiled by n^d patches is one big patch of n p volumes per
axis, whose update the single-patch definition fixes.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2306_16731_amd import workloads as wl
from tests import invariants as inv

GAMMA = wl.GAMMA


def _block(coord, p, dim):
    """Slices of the big patch's padded array holding the interior of the patch at grid coord."""
    sl = [slice(1 + c * p, 1 + (c + 1) * p) for c in coord]
    return tuple(reversed(sl))  # arrays are indexed [k, j, i]


def big_patch(mesh: wl.Mesh, data: np.ndarray) -> np.ndarray:
    """The n p-volume patch the mesh tiles: interiors copied block by block; face halos
    wrapped (periodic) or taken from the patches' own halos on the domain boundary."""
    b = mesh.batch
    p, dim, nq, n = int(b.sizes[0]), b.dim, b.nq, mesh.n
    P = n * p
    big = np.zeros((P + 2,) * dim + (nq,))
    for t in range(b.num_patches):
        v = inv.patch_view(data, int(b.offsets[t]), p, dim, nq)
        big[_block(mesh.coords[t], p, dim)] = inv.interior(v, dim)
    if mesh.periodic:
        inv.periodic_fill(big, dim)
        return big
    # boundary faces: the big patch's halo volume next to a boundary patch is that patch's halo volume
    for t in range(b.num_patches):
        v = inv.patch_view(data, int(b.offsets[t]), p, dim, nq)
        c = mesh.coords[t]
        for a in range(dim):
            for s in (0, 1):
                if mesh.neighbors[t, 2 * a + s] >= 0:
                    continue
                # array axis of grid axis a is dim - 1 - a
                ax = dim - 1 - a
                src = [slice(1, p + 1)] * dim
                dst = list(_block(c, p, dim))
                src[ax] = 0 if s == 0 else p + 1
                dst[ax] = 0 if s == 0 else P + 1
                big[tuple(dst)] = v[tuple(src)]
    return big


def check_big_patch_equivalence(update, n, p, dim, periodic, nq=5, seed=0, tol=0.0, dt=1.3e-3):
    """One mesh step equals one step of the big patch the mesh tiles, volume by volume; each
    patch's lambda is the maximum over its new interior (computed with numpy)."""
    mesh = wl.make_mesh(n, p, dim=dim, nq=nq, seed=seed, periodic=periodic)
    b = mesh.batch
    T = b.num_patches
    h = mesh.h
    out, lam = update(b.data, b.sizes, b.offsets, mesh.neighbors, dim, nq, np.full(T, dt), np.full(T, h))
    big = big_patch(mesh, b.data)
    P = n * p
    want, _ = oracle.batch_update(big.reshape(-1), [P], [0], dim, nq, dt, h, GAMMA, False)
    want = want.reshape(big.shape)
    for t in range(T):
        got_t = inv.interior(inv.patch_view(out, int(b.offsets[t]), p, dim, nq), dim)
        want_t = want[_block(mesh.coords[t], p, dim)]
        if tol == 0.0:
            assert np.array_equal(got_t, want_t), (n, p, dim, periodic, t)
        else:
            assert inv.rel_err(got_t, want_t) <= tol, (n, p, dim, periodic, t, inv.rel_err(got_t, want_t))
    ref_lam = inv.independent_lambda(out, b.sizes, b.offsets, dim, nq)
    np.testing.assert_allclose(lam, ref_lam, rtol=max(tol, 1e-14), atol=0)
    return mesh, out, lam


def check_fill_leaves_the_rest(fill, n, p, dim, periodic, nq=5, seed=1):
    """The fill writes face halos only (corner / edge halos and interiors unchanged), and a
    halo volume on a boundary face without a neighbour keeps its value."""
    mesh = wl.make_mesh(n, p, dim=dim, nq=nq, seed=seed, periodic=periodic)
    b = mesh.batch
    got = fill(b.data, b.sizes, b.offsets, mesh.neighbors, dim, nq)
    face = inv.face_halo_mask(p, dim)
    inner = np.zeros_like(face)
    inner[(slice(1, -1),) * dim] = True
    for t in range(b.num_patches):
        g = inv.patch_view(got, int(b.offsets[t]), p, dim, nq)
        d = inv.patch_view(b.data, int(b.offsets[t]), p, dim, nq)
        assert np.array_equal(g[~face], d[~face]), "corner / edge halo written"
        assert np.array_equal(g[inner], d[inner]), "interior written"
        for a in range(dim):
            ax = dim - 1 - a
            for s in (0, 1):
                nbt = mesh.neighbors[t, 2 * a + s]
                sl = [slice(1, p + 1)] * dim
                sl[ax] = 0 if s == 0 else p + 1
                if nbt < 0:
                    assert np.array_equal(g[tuple(sl)], d[tuple(sl)]), "boundary halo changed"
                else:
                    src = [slice(1, p + 1)] * dim
                    src[ax] = p if s == 0 else 1
                    nv = inv.patch_view(b.data, int(b.offsets[nbt]), p, dim, nq)
                    assert np.array_equal(g[tuple(sl)], nv[tuple(src)]), (t, a, s)


def check_per_patch_step_sizes(update_lts, p, dim, T=6, nq=5, seed=2, tol=0.0):
    """With its own dt and h, every patch advances exactly as it would alone (the
    single-patch definition with scalar dt and h)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    data, sizes, offsets = inv.random_batch(rng, T, p, dim, nq)
    dt = rng.uniform(0.5e-3, 2e-3, T)
    h = rng.uniform(1 / 64, 1 / 32, T)
    out, lam = update_lts(data, sizes, offsets, dim, nq, dt, h)
    for t in range(T):
        n = (p + 2) ** dim * nq
        one = data[offsets[t]:offsets[t] + n].copy()
        want, wl_ = oracle.batch_update(one, [p], [0], dim, nq, float(dt[t]), float(h[t]), GAMMA, False)
        if tol == 0.0:
            assert np.array_equal(out[offsets[t]:offsets[t] + n], want), t
            assert lam[t] == wl_[0], t
        else:
            assert inv.rel_err(out[offsets[t]:offsets[t] + n], want) <= tol, t
            assert abs(lam[t] - wl_[0]) <= tol * wl_[0], t


def check_local_dt(local_dt, T=50, seed=3, tol=0.0):
    """Per-patch step sizes: with one h, the smallest equals the global step size
    cfl h / (d max lambda) (division rounds monotonically); each patch's Courant
    number d lambda dt / h equals cfl to rounding."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = rng.uniform(0.5, 3.0, T)
    for dim in (2, 3):
        h = 1.0 / 48.0
        dt = local_dt(lam, np.full(T, h), dim, wl.CFL)
        glob = wl.CFL * h / (dim * np.max(lam))
        if tol == 0.0:
            assert np.min(dt) == glob
        else:
            assert abs(np.min(dt) - glob) <= tol * glob
        hv = rng.uniform(1 / 64, 1 / 16, T)
        dtv = local_dt(lam, hv, dim, wl.CFL)
        np.testing.assert_allclose(dim * lam * dtv / hv, wl.CFL, rtol=4e-16 + tol, atol=0)
