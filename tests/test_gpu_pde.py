"""The generic solver of Eq. 1 on the GPU through fv_pde_batch_update (needs a gfx950
GPU): every built-in PDE against the CPU oracle element by element (1e-12
relative per unknown, as elsewhere), and the pins of tests/pde_checks.py run on
the HIP path."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2306_16731_amd import workloads as wl
from tests import hip_path as hp
from tests import pde_checks as pc

pytestmark = pytest.mark.gpu
TOL = 1e-12
OIDS = {"euler": oracle.PDE_EULER, "shallow_water": oracle.PDE_SHALLOW_WATER, "advection": oracle.PDE_ADVECTION,
        "acoustics": oracle.PDE_ACOUSTICS, "acoustics_ncp": oracle.PDE_ACOUSTICS_NCP}


def _announce(msg):
    print(f"[gpu-pde] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16731_amd import fvpatch
    fvpatch.load()


def gpu_update(name, prm, data, sizes, offsets, dim, dt, h, periodic, pass_offsets=True):
    import torch
    from paper_2306_16731_amd import fvpatch
    a = hp.to_dev(np.asarray(data, np.float64))
    b = a.clone()
    T = len(sizes)
    lam = torch.full((T,), -1.0, dtype=torch.float64, device="cuda")
    fvpatch.fv_pde_batch_update(fvpatch.PDE_IDS[name], prm, a, b, np.asarray(sizes, np.int32),
                                np.asarray(offsets, np.int64) if pass_offsets else None, T, dim, dt, h,
                                fvpatch.FV_HALO_PERIODIC if periodic else 0, lam)
    torch.cuda.synchronize()
    return b.cpu().numpy(), lam.cpu().numpy()


def gpu_fill(data, sizes, offsets, nb, dim, nq):
    import torch
    from paper_2306_16731_amd import fvpatch
    mesh = fvpatch.fv_mesh_create(sizes, offsets, nb, len(sizes), dim, nq)
    try:
        d = hp.to_dev(np.asarray(data, np.float64))
        fvpatch.fv_mesh_halo_fill(mesh, d)
        torch.cuda.synchronize()
        return d.cpu().numpy()
    finally:
        fvpatch.fv_mesh_destroy(mesh)


def compare(name, dim, b, dt, h, periodic, pass_offsets=True):
    got, lam = gpu_update(name, pc.PRM[name], b.data, b.sizes, b.offsets, dim, dt, h, periodic, pass_offsets)
    want, wlam = oracle.pde_update(OIDS[name], pc.PRM[name], b.data, b.sizes, b.offsets, dim, dt, h, periodic)
    err = hp.component_errors(got, want, b.nq)
    assert np.all(err <= TOL), (name, dim, err)
    assert hp.lambda_error(lam, wlam) <= TOL, hp.lambda_error(lam, wlam)
    return got, lam


CASES = [  # (name, dim, sizes)
    ("shallow_water", 2, [16] * 9),
    ("shallow_water", 2, [3, 17, 5, 64, 9, 1, 31]),
    ("advection", 2, [8] * 11),
    ("advection", 2, [16] * 7),                 # the 2D wave form (p = 16, 16-byte bursts when periodic)
    ("acoustics", 2, [16] * 4 + [7]),           # wave form and plane-marching kernel in one batch
    ("advection", 3, [4, 7, 12, 24, 1, 5]),
    ("acoustics", 2, [9, 33, 2, 62]),
    ("acoustics", 3, [6] * 7 + [13]),
    ("acoustics_ncp", 2, [16, 5, 63]),
    ("acoustics_ncp", 3, [8, 3, 23, 10]),   # 23: the largest 3D size whose block fits the LDS
    ("advection", 3, [8] * 5 + [4] * 3),         # the 3D interior-mapped form (p = 4, 8)
    ("acoustics", 3, [4] * 9 + [8] * 3 + [5]),   # interior-mapped form and plane-marching kernel in one batch
    ("acoustics_ncp", 3, [4] * 6 + [8] * 2),
    ("shallow_water", 2, [3] * 23 + [5] * 9 + [9] * 8 + [17] * 5),   # the 2D wave form at every fixed size
    ("acoustics_ncp", 2, [17] * 5 + [9] * 7 + [3] * 3),
    ("advection", 2, [5] * 12 + [3] * 40 + [17] * 2),
    ("euler", 2, [16, 7, 40]),
    ("euler", 3, [8, 5]),
]


@pytest.mark.parametrize("name,dim,sizes", CASES)
@pytest.mark.parametrize("periodic", [False, True])
def test_pde_matches_oracle(name, dim, sizes, periodic):
    _announce(f"{name} dim={dim} sizes={sizes} periodic={periodic}")
    b = wl.make_pde_batch(name, sizes, dim=dim, seed=len(sizes) + dim)
    compare(name, dim, b, 1.7e-3, 1.0 / 40, periodic)


@pytest.mark.parametrize("name,dim", [("shallow_water", 2), ("acoustics", 3)])
def test_contiguous_and_gapped_layouts(name, dim):
    """Offsets NULL (contiguous) and patches at gapped, odd offsets give the same results;
    the gaps are not written."""
    _announce(f"layouts {name} dim={dim}")
    p, T = 12 if dim == 2 else 6, 10
    b = wl.make_pde_batch(name, [p] * T, dim=dim, seed=3)
    got_c, lam_c = compare(name, dim, b, 1e-3, 1.0 / 30, False, pass_offsets=False)
    n = (p + 2) ** dim * b.nq
    rng = np.random.Generator(np.random.PCG64(4))
    starts = np.cumsum(np.concatenate([[3], n + rng.integers(1, 6, size=T - 1)])).astype(np.int64)
    data = rng.uniform(-1, 1, int(starts[-1] + n + 5))
    for t in range(T):
        data[starts[t]:starts[t] + n] = b.data[b.offsets[t]:b.offsets[t] + n]
    got, lam = gpu_update(name, pc.PRM[name], data, b.sizes, starts, dim, 1e-3, 1.0 / 30, False)
    inside = np.zeros(len(data), bool)
    for t in range(T):
        assert np.array_equal(got[starts[t]:starts[t] + n], got_c[b.offsets[t]:b.offsets[t] + n])
        inside[starts[t]:starts[t] + n] = True
    assert np.array_equal(got[~inside], data[~inside])
    assert np.array_equal(lam, lam_c)


def test_euler_through_the_generic_entry_is_the_euler_path():
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce("euler via fv_pde_batch_update")
    for dim, p in ((2, 16), (2, 7), (3, 8)):
        b = wl.make_uniform(20, p, dim=dim, seed=p)
        got, lam = gpu_update("euler", [wl.GAMMA], b.data, b.sizes, b.offsets, dim, 1e-3, wl.H_DEFAULT, True)
        want, wlam = hp.gpu_step(b.data, b.sizes, b.offsets, dim, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, True)
        assert np.array_equal(got, want) and np.array_equal(lam, wlam)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dim", [2, 3])
def test_advection_is_upwind(dim):
    _announce(f"advection upwind {dim}D")
    pc.check_advection_is_upwind(gpu_update, dim)


@pytest.mark.parametrize("name", ["advection", "acoustics", "acoustics_ncp"])
@pytest.mark.parametrize("dim", [2, 3])
def test_fourier_mode(name, dim):
    _announce(f"fourier {name} {dim}D")
    pc.check_fourier_mode(gpu_update, name, dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_ncp_form_equals_flux_form(dim):
    _announce(f"ncp form {dim}D")
    pc.check_ncp_form_equals_flux_form(gpu_update, dim)


@pytest.mark.parametrize("p", [16, 5, 10])   # the 2D wave form (even and odd rows) and the plane-marching kernel
def test_shallow_water_pins(p):
    _announce(f"lake at rest / conservation / swap / coriolis p={p}")
    pc.check_lake_at_rest(gpu_update, p=p)
    pc.check_swe_conservation(gpu_update, p=p)
    pc.check_swe_swap_xy(gpu_update, p=p)
    pc.check_coriolis(gpu_update, p=p)


@pytest.mark.parametrize("name", ["advection", "acoustics", "acoustics_ncp"])
@pytest.mark.parametrize("p", [8, 4])
def test_fourier_mode_3d_interior_form(name, p):
    _announce(f"fourier {name} 3D p={p}")
    pc.check_fourier_mode(gpu_update, name, 3, p=p, modes=((1, 2, 3), (3, 1, 2), (p // 2, p // 2, 0)))


@pytest.mark.parametrize("name", ["advection", "acoustics", "acoustics_ncp"])
@pytest.mark.parametrize("p", [16, 9])
def test_fourier_mode_wave_form(name, p):
    _announce(f"fourier {name} 2D p={p}")
    pc.check_fourier_mode(gpu_update, name, 2, p=p, modes=((1, 2, 0), (3, p // 3, 0), (p // 2, p // 2, 0)))


def test_dam_break_converges_to_stoker():
    _announce("dam break")
    errs = pc.check_dam_break_converges(gpu_update, gpu_fill, resolutions=(64, 128, 256))
    print("L1 errors", errs)


def test_errors():
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce("errors")
    a = torch.zeros(10000, dtype=torch.float64, device="cuda")
    c = torch.zeros_like(a)
    sz = np.array([4], np.int32)

    def call(pde, prm, dim=2, **kw):
        return fvpatch.fv_pde_batch_update(pde, prm, a, c, sz, None, 1, dim, 1e-3, 0.1, raise_on_error=False, **kw)

    assert call(fvpatch.FV_PDE_SHALLOW_WATER, [9.81, 0.0], dim=3) == fvpatch.FV_ERR_UNSUPPORTED
    assert call(fvpatch.FV_PDE_SHALLOW_WATER, [9.81]) == fvpatch.FV_ERR_INVALID_ARG
    assert call(fvpatch.FV_PDE_SHALLOW_WATER, [-1.0, 0.0]) == fvpatch.FV_ERR_INVALID_ARG
    assert call(fvpatch.FV_PDE_ACOUSTICS, [0.0, 1.0]) == fvpatch.FV_ERR_INVALID_ARG
    assert call(fvpatch.FV_PDE_ADVECTION, [1.0, np.nan, 0.0]) == fvpatch.FV_ERR_INVALID_ARG
    assert call(9, [1.0]) == fvpatch.FV_ERR_INVALID_ARG
    assert fvpatch.fv_pde_batch_update(fvpatch.FV_PDE_ADVECTION, [1.0, 0.0, 0.0], a, a, sz, None, 1, 2, 1e-3, 0.1,
                                       raise_on_error=False) == fvpatch.FV_ERR_OVERLAP
    assert call(fvpatch.FV_PDE_ADVECTION, [1.0, 0.0, 0.0]) == fvpatch.FV_OK
    big = torch.zeros(26 ** 3 * 4, dtype=torch.float64, device="cuda")
    assert fvpatch.fv_pde_batch_update(fvpatch.FV_PDE_ACOUSTICS_NCP, [1.0, 1.0], big, big.clone(),
                                       np.array([24], np.int32), None, 1, 3, 1e-3, 0.1,
                                       raise_on_error=False) == fvpatch.FV_ERR_UNSUPPORTED
    torch.cuda.synchronize()
