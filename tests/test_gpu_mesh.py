"""Patch-mesh steps on the GPU through the C ABI (needs a gfx950 GPU): the face-halo
fill, the fused mesh step (halos read from the neighbours, per-patch dt and h)
and the per-patch step sizes, against the pins of tests/mesh_checks.py and the
CPU oracle.  Tolerance as elsewhere: 1e-12 relative; the fill is a copy and
must be exact."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2306_16731_amd import workloads as wl
from tests import hip_path as hp
from tests import invariants as inv
from tests import mesh_checks as mc

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _announce(msg):
    print(f"[gpu-mesh] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16731_amd import fvpatch
    fvpatch.load()


def gpu_fill(data, sizes, offsets, nb, dim, nq, pass_offsets=True):
    import torch
    from paper_2306_16731_amd import fvpatch
    T = len(sizes)
    mesh = fvpatch.fv_mesh_create(sizes, offsets if pass_offsets else None, nb, T, dim, nq)
    try:
        d = hp.to_dev(np.asarray(data, np.float64))
        fvpatch.fv_mesh_halo_fill(mesh, d)
        torch.cuda.synchronize()
        return d.cpu().numpy()
    finally:
        fvpatch.fv_mesh_destroy(mesh)


def gpu_update(data, sizes, offsets, nb, dim, nq, dt, h, pass_offsets=True):
    import torch
    from paper_2306_16731_amd import fvpatch
    T = len(sizes)
    mesh = fvpatch.fv_mesh_create(sizes, offsets if pass_offsets else None, nb, T, dim, nq)
    try:
        a = hp.to_dev(np.asarray(data, np.float64))
        b = a.clone()
        ddt = hp.to_dev(np.asarray(dt, np.float64))
        dh = hp.to_dev(np.asarray(h, np.float64))
        lam = torch.full((T,), -1.0, dtype=torch.float64, device="cuda")
        fvpatch.fv_mesh_step(mesh, a, b, ddt, dh, wl.GAMMA, lam)
        torch.cuda.synchronize()
        return b.cpu().numpy(), lam.cpu().numpy()
    finally:
        fvpatch.fv_mesh_destroy(mesh)


def gpu_local_dt(lam, h, dim, cfl):
    import torch
    from paper_2306_16731_amd import fvpatch
    dl = hp.to_dev(np.asarray(lam, np.float64))
    dh = hp.to_dev(np.asarray(h, np.float64))
    out = torch.empty_like(dl)
    fvpatch.fv_local_dt(dl, dh, len(lam), dim, cfl, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,p,dim,periodic", [(3, 4, 2, True), (4, 7, 2, False), (3, 16, 2, True), (2, 5, 3, True),
                                              (3, 3, 3, False)])
def test_fill_matches_oracle_exactly(n, p, dim, periodic):
    _announce(f"fill n={n} p={p} dim={dim} periodic={periodic}")
    mc.check_fill_leaves_the_rest(gpu_fill, n, p, dim, periodic)
    m = wl.make_mesh(n, p, dim=dim, seed=4, periodic=periodic)
    b = m.batch
    want = oracle.halo_fill(b.data, b.sizes, b.offsets, m.neighbors, dim, 5)
    assert np.array_equal(gpu_fill(b.data, b.sizes, b.offsets, m.neighbors, dim, 5, pass_offsets=False), want)


MESH_CASES = [(3, 3, 2, True), (3, 5, 2, False), (2, 9, 2, True), (4, 16, 2, True), (2, 16, 2, False),
              (2, 17, 2, True), (2, 4, 3, True), (2, 6, 3, False), (2, 8, 3, True), (3, 8, 3, False)]


@pytest.mark.parametrize("n,p,dim,periodic", MESH_CASES)
def test_mesh_step_equals_big_patch(n, p, dim, periodic):
    """The fused mesh step (halos read from the neighbours during the update) against the
    oracle's step of the one big patch the mesh tiles."""
    _announce(f"mesh step n={n} p={p} dim={dim} periodic={periodic}")
    mc.check_big_patch_equivalence(gpu_update, n, p, dim, periodic, tol=TOL)


@pytest.mark.parametrize("n,p,dim", [(4, 16, 2), (3, 9, 2), (2, 8, 3), (3, 4, 3)])
def test_fused_step_is_fill_then_plain_update_bitwise(n, p, dim):
    """Reading halos from the neighbours inside the kernel gives bit for bit what a separate
    fill followed by the plain launch gives (same dt / h for every patch), with patches at
    gapped offsets."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"fused vs fill + plain n={n} p={p} dim={dim}")
    m = wl.make_mesh(n, p, dim=dim, seed=5, periodic=True)
    b = m.batch
    T = b.num_patches
    vol = (p + 2) ** dim * 5
    rng = np.random.Generator(np.random.PCG64(6))
    starts = np.cumsum(np.concatenate([[2], vol + 2 * rng.integers(0, 3, size=T - 1)])).astype(np.int64)
    data = rng.uniform(-1, 1, int(starts[-1] + vol + 2))
    for t in range(T):
        data[starts[t]:starts[t] + vol] = b.data[b.offsets[t]:b.offsets[t] + vol]
    dt, h = 1.1e-3, m.h
    fused, lam_f = gpu_update(data, b.sizes, starts, m.neighbors, dim, 5, np.full(T, dt), np.full(T, h))
    filled = gpu_fill(data, b.sizes, starts, m.neighbors, dim, 5)
    plain, lam_p = hp.gpu_step(filled, b.sizes, starts, dim, 5, dt, h, wl.GAMMA, False)
    inside = np.zeros(len(data), bool)
    for t in range(T):
        v = np.zeros(vol, bool).reshape((p + 2,) * dim + (5,))
        v[(slice(1, -1),) * dim] = True
        inside[starts[t]:starts[t] + vol] = v.reshape(-1)
    assert np.array_equal(fused[inside], plain[inside])
    assert np.array_equal(lam_f, lam_p)
    assert np.array_equal(fused[~inside], data[~inside]), "the mesh step wrote outside the interiors"


@pytest.mark.parametrize("p,dim", [(16, 2), (5, 2), (8, 3)])
def test_per_patch_step_sizes(p, dim):
    """Every patch with its own dt and h (no neighbours: own halos) advances as the
    single-patch oracle with that dt and h."""
    _announce(f"per-patch dt / h p={p} dim={dim}")

    def update_lts(data, sizes, offsets, dim_, nq, dt, h):
        nb = np.full((len(sizes), 2 * dim_), -1, np.int32)
        return gpu_update(data, sizes, offsets, nb, dim_, nq, dt, h)

    mc.check_per_patch_step_sizes(update_lts, p, dim, T=7, tol=TOL)


def test_local_dt():
    _announce("local dt")
    mc.check_local_dt(gpu_local_dt)


def test_mesh_errors():
    import torch
    from paper_2306_16731_amd import fvpatch
    m = wl.make_mesh(2, 7, dim=2, periodic=True)
    b = m.batch
    mesh = fvpatch.fv_mesh_create(b.sizes, None, m.neighbors, b.num_patches, 2, 5)
    try:
        a = hp.to_dev(b.data)
        c = a.clone()
        dt = torch.full((b.num_patches,), 1e-3, dtype=torch.float64, device="cuda")
        # p = 7 has no fixed-size build: the fused step is refused, the fill works
        assert fvpatch.fv_mesh_step(mesh, a, c, dt, dt, 1.4, None, raise_on_error=False) == fvpatch.FV_ERR_UNSUPPORTED
        assert fvpatch.fv_mesh_halo_fill(mesh, a, raise_on_error=False) == fvpatch.FV_OK
        torch.cuda.synchronize()
    finally:
        fvpatch.fv_mesh_destroy(mesh)
    m = wl.make_mesh(2, 16, dim=2, periodic=True)
    b = m.batch
    mesh = fvpatch.fv_mesh_create(b.sizes, None, m.neighbors, b.num_patches, 2, 5)
    try:
        a = hp.to_dev(b.data)
        dt = torch.full((b.num_patches,), 1e-3, dtype=torch.float64, device="cuda")
        assert fvpatch.fv_mesh_step(mesh, a, a, dt, dt, 1.4, None, raise_on_error=False) == fvpatch.FV_ERR_OVERLAP
        assert fvpatch.fv_mesh_step(mesh, a, a.clone(), None, dt, 1.4, None,
                                    raise_on_error=False) == fvpatch.FV_ERR_INVALID_ARG
    finally:
        fvpatch.fv_mesh_destroy(mesh)
