"""Pins of the generic solver of Eq. 1 (flux, non-conservative product, source,
wave speed supplied per PDE) and of the PDEs built on it.

Every check takes the implementation under test as a callable, so the same pins
hold the CPU oracle (tests/test_oracle_pde.py) and the HIP path
(tests/test_gpu_pde.py):

    update(name, prm, data, sizes, offsets, dim, dt, h, periodic) -> (out, lambda)
        one explicit Euler step of every patch of the PDE `name` (a name of
        workloads.PDE_NAMES) with parameters prm; ``out`` starts as a copy of data.
    terms(name, dim, prm, q, n, dq) -> (F_n(q), lambda_n(q), B_n(q) dq, S(q))
        (oracle only) the user terms of one volume.

What fixes the expected values is never the code under test:
  - linear advection: the step is the textbook upwind scheme;
  - linear acoustics: every Fourier mode is multiplied by the scheme's
    amplification matrix, worked out by hand from the update formula and
    Eq. 2; the system written with the non-conservative product gives the same
    step as written with the flux;
  - shallow water: lambda_n is the largest eigenvalue magnitude of the
    quasi-linear matrix dF_n/dQ + B_n; a lake at rest keeps zero momentum;
    mass is conserved on periodic patches; mirroring x and y commutes with the
    step; Coriolis deflects a flow to the right of its motion for f > 0; and
    a dam break converges, under refinement, to Stoker's exact solution.
"""
from __future__ import annotations

import numpy as np

from paper_2306_16731_amd import workloads as wl
from tests import invariants as inv

PRM = {name: wl.default_params(name) for name in wl.PDE_NAMES}


def _single_periodic_patch(vols: np.ndarray, dim: int):
    """A batch of one patch from interior states [p]*dim + [nq], its face halos wrapped."""
    p = vols.shape[0]
    nq = vols.shape[-1]
    full = np.zeros((p + 2,) * dim + (nq,))
    full[(slice(1, -1),) * dim] = vols
    inv.periodic_fill(full, dim)
    return full.reshape(-1).copy(), np.array([p], np.int32), np.array([0], np.int64)


def _interior(data, p, dim, nq):
    return inv.interior(inv.patch_view(data, 0, p, dim, nq), dim)


# ---------------------------------------------------------------- linear PDEs: closed forms
def check_advection_is_upwind(update, dim, p=9, seed=0, tol=1e-14):
    """Rusanov's flux with lambda = |a_n| is the upwind value a_n q_upwind, so one step is the
    upwind scheme q + r sum_n a_n (q_(c - s e_n) - q_c) s  with s = sign(a_n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = np.array(PRM["advection"][:dim])
    q = rng.uniform(-1, 1, (p,) * dim + (1,))
    data, sizes, offsets = _single_periodic_patch(q, dim)
    dt, h = 0.01, 1.0 / 32
    r = dt / h
    out, lam = update("advection", PRM["advection"], data, sizes, offsets, dim, dt, h, False)
    want = q[..., 0].copy()
    for n in range(dim):
        ax = dim - 1 - n
        s = 1 if a[n] > 0 else -1
        upwind = np.roll(q[..., 0], s, axis=ax)   # q at c - s e_n (periodic)
        want = want + r * a[n] * (upwind - q[..., 0]) * s
    got = _interior(out, p, dim, 1)[..., 0]
    assert inv.rel_err(got, want) <= tol, inv.rel_err(got, want)
    assert lam[0] == np.max(np.abs(a))


def acoustic_matrices(dim, rho0, K0):
    """A_n of linear acoustics, Q = (p, u_1 .. u_d): dp/dt + K0 du_n/dx_n = 0,
    du_n/dt + (1 / rho0) dp/dx_n = 0."""
    mats = []
    for n in range(dim):
        A = np.zeros((1 + dim, 1 + dim))
        A[0, 1 + n] = K0
        A[1 + n, 0] = 1.0 / rho0
        mats.append(A)
    return mats


def check_fourier_mode(update, name, dim, p=12, modes=((1, 2, 3), (3, 5, 1), (6, 0, 2)), seed=1, tol=1e-13):
    """One step of a periodic Fourier mode Re(Qhat exp(i theta . x)) of a linear system with
    constant wave speed c gives Re(M Qhat exp(i theta . x)), where, from the update formula and
    Eq. 2 with Q_(c +- e_n) = exp(+- i theta_n) Q_c,
        M = I + (dt/h) sum_n ( -i sin(theta_n) A_n + c (cos(theta_n) - 1) I )."""
    rng = np.random.Generator(np.random.PCG64(seed))
    prm = PRM[name]
    if name == "advection":
        A = [np.array([[prm[n]]]) for n in range(dim)]
        speeds = [abs(prm[n]) for n in range(dim)]
    else:
        A = acoustic_matrices(dim, prm[0], prm[1])
        speeds = [np.sqrt(prm[1] / prm[0])] * dim
    nq = A[0].shape[0]
    dt, h = 0.004, 1.0 / 24
    r = dt / h
    for k in modes:
        theta = [2 * np.pi * k[n] / p for n in range(dim)]
        qhat = rng.normal(size=nq) + 1j * rng.normal(size=nq)
        idx = np.indices((p,) * dim)            # idx[ax] over array axes (k, j, i)
        phase = sum(theta[n] * idx[dim - 1 - n] for n in range(dim))
        wave = np.exp(1j * phase)[..., None]
        q = np.real(qhat * wave)
        data, sizes, offsets = _single_periodic_patch(q, dim)
        out, _ = update(name, prm, data, sizes, offsets, dim, dt, h, False)
        M = np.eye(nq, dtype=complex)
        for n in range(dim):
            M = M + r * (-1j * np.sin(theta[n]) * A[n] + speeds[n] * (np.cos(theta[n]) - 1.0) * np.eye(nq))
        want = np.real((M @ qhat) * wave)
        got = _interior(out, p, dim, nq)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert err <= tol, (name, dim, k, err)


def check_ncp_form_equals_flux_form(update, dim, p=7, T=3, seed=2, tol=1e-13):
    """Linear acoustics written with the non-conservative product B_n = A_n (and F = 0)
    steps like the same system written with the flux F_n = A_n Q: the central jump terms
    sum to the central flux difference."""
    b = wl.make_pde_batch("acoustics", np.full(T, p), dim=dim, seed=seed)
    dt, h = 0.003, 1.0 / 20
    a, la = update("acoustics", PRM["acoustics"], b.data, b.sizes, b.offsets, dim, dt, h, True)
    c, lc = update("acoustics_ncp", PRM["acoustics_ncp"], b.data, b.sizes, b.offsets, dim, dt, h, True)
    assert inv.rel_err(c, a) <= tol, inv.rel_err(c, a)
    assert np.array_equal(la, lc)


# ---------------------------------------------------------------- shallow water
def swe_state(h, u, v, b):
    return np.stack(np.broadcast_arrays(h, h * u, h * v, b), axis=-1).astype(np.float64)


def check_swe_eigenvalue(terms, samples=20, seed=3, tol=1e-6):
    """lambda_n equals the largest eigenvalue magnitude of dF_n/dQ + B_n(Q) over the evolved
    unknowns (the Jacobian by central differences, B_n column by column)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    prm = PRM["shallow_water"]
    for _ in range(samples):
        q = swe_state(rng.uniform(0.5, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0, 1))
        for n in range(2):
            J = np.zeros((3, 3))
            for k in range(3):
                e = np.zeros(4)
                eps = 1e-6 * max(1.0, abs(q[k]))
                e[k] = eps
                fp = terms("shallow_water", 2, prm, q + e, n, np.zeros(4))[0]
                fm = terms("shallow_water", 2, prm, q - e, n, np.zeros(4))[0]
                J[:, k] = (fp - fm) / (2 * eps)
                unit = np.zeros(4)
                unit[k] = 1.0
                J[:, k] += terms("shallow_water", 2, prm, q, n, unit)[2]
            lam = terms("shallow_water", 2, prm, q, n, np.zeros(4))[1]
            ev = np.max(np.abs(np.linalg.eigvals(J)))
            assert abs(ev - lam) <= tol * lam, (q, n, ev, lam)


def check_lake_at_rest(update, p=10, T=2, seed=4):
    """Still water over an uneven bottom (h + b constant, no velocity): the hydrostatic
    non-conservative product balances exactly, so the momentum stays zero, bit for bit.  (The
    depth itself moves by the Rusanov dissipation of its jumps: the scheme is not
    well-balanced, as plain Rusanov is not.)  A flat lake does not change at all."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nvol = (p + 2) ** 2
    for flat in (False, True):
        vols = []
        for _ in range(T):
            # dyadic depths and bottoms: h + b is exactly 1.5 and every jump of h cancels the jump of b
            b = np.zeros(nvol) if flat else rng.integers(0, 33, nvol) / 64.0
            vols.append(swe_state(1.5 - b, 0.0, 0.0, b))
        data = np.concatenate(vols).reshape(-1)
        sizes = np.full(T, p, np.int32)
        offsets = np.arange(T, dtype=np.int64) * nvol * 4
        prm = [wl.SWE_G, 0.0]
        out, lam = update("shallow_water", prm, data, sizes, offsets, 2, 2e-3, 1.0 / 40, False)
        for t in range(T):
            g = inv.interior(inv.patch_view(out, int(offsets[t]), p, 2, 4), 2)
            d = inv.interior(inv.patch_view(data, int(offsets[t]), p, 2, 4), 2)
            assert np.all(g[..., 1:3] == 0.0), "momentum of a lake at rest changed"
            assert np.array_equal(g[..., 3], d[..., 3]), "bathymetry changed"
            if flat:
                assert np.array_equal(g, d), "flat lake at rest changed"
            np.testing.assert_allclose(lam[t], np.max(np.sqrt(wl.SWE_G * g[..., 0])), rtol=1e-15)


def check_swe_conservation(update, p=9, T=3, seed=5, tol=1e-13):
    """Periodic patches: the sum of the depth over each interior is conserved.  Over a flat
    bottom without Coriolis the momentum sums are conserved too: with the face average of the
    depth, g hbar (h_R - h_L) = g h_R^2 / 2 - g h_L^2 / 2, so the hydrostatic non-conservative
    product is the conservative pressure flux and telescopes over a periodic patch."""
    for flat in (False, True):
        b = wl.make_pde_batch("shallow_water", np.full(T, p), dim=2, seed=seed)
        prm = list(PRM["shallow_water"])
        if flat:
            b.data.reshape(-1, 4)[:, 3] = 0.25
            prm[1] = 0.0
        for t in range(T):
            inv.periodic_fill(inv.patch_view(b.data, int(b.offsets[t]), p, 2, 4), 2)
        out, _ = update("shallow_water", prm, b.data, b.sizes, b.offsets, 2, 2e-3, 1.0 / 30, True)
        for t in range(T):
            s0 = np.sum(inv.interior(inv.patch_view(b.data, int(b.offsets[t]), p, 2, 4), 2), axis=(0, 1))
            s1 = np.sum(inv.interior(inv.patch_view(out, int(b.offsets[t]), p, 2, 4), 2), axis=(0, 1))
            assert abs(s1[0] - s0[0]) <= tol * s0[0], (s0, s1)
            if flat:
                scale = np.sum(np.abs(inv.interior(inv.patch_view(b.data, int(b.offsets[t]), p, 2, 4), 2)[..., 1:3]))
                assert np.all(np.abs(s1[1:3] - s0[1:3]) <= tol * scale), (s0, s1)


def check_swe_swap_xy(update, p=8, seed=6):
    """Swapping x and y (with hu and hv) commutes with the step bit for bit (no Coriolis:
    rotation by f has a handedness)."""
    b = wl.make_pde_batch("shallow_water", [p], dim=2, seed=seed)
    prm = [wl.SWE_G, 0.0]
    view = inv.patch_view(b.data, 0, p, 2, 4)
    sw = np.swapaxes(view, 0, 1).copy()
    sw[..., [1, 2]] = sw[..., [2, 1]]
    out, lam = update("shallow_water", prm, b.data, b.sizes, b.offsets, 2, 2e-3, 1.0 / 30, False)
    out_s, lam_s = update("shallow_water", prm, sw.reshape(-1).copy(), b.sizes, b.offsets, 2, 2e-3, 1.0 / 30,
                          False)
    back = np.swapaxes(inv.patch_view(out_s, 0, p, 2, 4), 0, 1).copy()
    back[..., [1, 2]] = back[..., [2, 1]]
    assert np.array_equal(inv.interior(back, 2), inv.interior(inv.patch_view(out, 0, p, 2, 4), 2))
    assert lam[0] == lam_s[0]


def check_coriolis(update, p=6, f=0.8, dt=0.01, tol=1e-14):
    """A uniform flow over a flat bottom (no flux differences, no jumps) changes only by
    the source: for f > 0 the momentum turns clockwise, i.e. to the right of the motion (the
    Coriolis deflection of the northern hemisphere), by the angle atan(f dt) of one explicit
    Euler step, its magnitude growing by sqrt(1 + (f dt)^2); the depth does not change."""
    m = np.array([0.6, -0.25])
    q = np.broadcast_to(np.array([1.3, m[0], m[1], 0.2]), (p + 2, p + 2, 4)).copy()
    data = q.reshape(-1).copy()
    out, _ = update("shallow_water", [wl.SWE_G, f], data, np.array([p], np.int32), np.array([0], np.int64), 2, dt,
                    1.0 / 20, False)
    g = inv.interior(inv.patch_view(out, 0, p, 2, 4), 2)
    mn = g[..., 1:3].reshape(-1, 2)
    assert np.all(g[..., 0] == 1.3) and np.all(g[..., 3] == 0.2)
    cross = m[0] * mn[:, 1] - m[1] * mn[:, 0]
    assert np.all(cross < 0), "Coriolis turned the flow to the left"
    ang = np.arctan2(-cross, mn @ m)
    assert np.allclose(ang, np.arctan(f * dt), rtol=tol * 100, atol=0)
    assert np.allclose(np.linalg.norm(mn, axis=1), np.linalg.norm(m) * np.sqrt(1 + (f * dt) ** 2), rtol=tol, atol=0)


def stoker_depth(x, t, x0, hl, hr, g=wl.SWE_G):
    """Exact depth of the dam break over a wet bed (Stoker): a rarefaction into the deep side
    and a shock into the shallow side, joined by a middle state (hm, um) that satisfies
        um = 2 (sqrt(g hl) - sqrt(g hm))              (left-going rarefaction)
        um = (hm - hr) sqrt(g (hm + hr) / (2 hm hr))  (right-going shock, Rankine-Hugoniot)."""
    from scipy.optimize import brentq
    cl = np.sqrt(g * hl)

    def gap(hm):
        return 2 * (cl - np.sqrt(g * hm)) - (hm - hr) * np.sqrt(g * (hm + hr) / (2 * hm * hr))

    hm = brentq(gap, hr, hl, xtol=1e-15, rtol=1e-15)
    cm = np.sqrt(g * hm)
    um = 2 * (cl - cm)
    s = hm * um / (hm - hr)
    xi = (np.asarray(x) - x0) / t
    out = np.where(xi < -cl, hl, np.where(xi < um - cm, (2 * cl - xi) ** 2 / (9 * g), np.where(xi < s, hm, hr)))
    return out, hm, um


def dam_break(update, fill, cells, p=8, t_end=0.04, hl=2.0, hr=1.0, cfl=0.4):
    """A row of cells / p patches over [0, 1] (the dam at 1/2), periodic in y, with
    transmissive ends; returns (cell centres, depth, x-velocity) at t_end."""
    n = cells // p
    T = n
    nb = np.full((T, 4), -1, np.int32)
    for t in range(T):
        nb[t, 0] = t - 1 if t > 0 else -1
        nb[t, 1] = t + 1 if t < T - 1 else -1
        nb[t, 2] = nb[t, 3] = t                    # periodic in y: the patch is its own neighbour
    h = 1.0 / cells
    xc = (np.arange(cells) + 0.5) * h
    vol = (p + 2) ** 2 * 4
    data = np.zeros(T * vol)
    sizes = np.full(T, p, np.int32)
    offsets = np.arange(T, dtype=np.int64) * vol
    for t in range(T):
        v = inv.patch_view(data, int(offsets[t]), p, 2, 4)
        x = xc[t * p:(t + 1) * p]
        v[1:-1, 1:-1, 0] = np.where(x < 0.5, hl, hr)[None, :]
    time, prm = 0.0, [wl.SWE_G, 0.0]
    while time < t_end - 1e-15:
        data = fill(data, sizes, offsets, nb, 2, 4)
        first = inv.patch_view(data, int(offsets[0]), p, 2, 4)
        last = inv.patch_view(data, int(offsets[-1]), p, 2, 4)
        first[1:-1, 0] = first[1:-1, 1]            # transmissive ends
        last[1:-1, p + 1] = last[1:-1, p]
        hmax = max(float(np.max(inv.patch_view(data, int(o), p, 2, 4)[1:-1, 1:-1, 0])) for o in offsets)
        umax = max(float(np.max(np.abs(inv.patch_view(data, int(o), p, 2, 4)[1:-1, 1:-1, 1]
                                       / inv.patch_view(data, int(o), p, 2, 4)[1:-1, 1:-1, 0]))) for o in offsets)
        dt = min(cfl * h / (umax + np.sqrt(wl.SWE_G * hmax)), t_end - time)
        data, _ = update("shallow_water", prm, data, sizes, offsets, 2, dt, h, False)
        time += dt
    depth = np.concatenate([inv.patch_view(data, int(o), p, 2, 4)[p // 2, 1:-1, 0] for o in offsets])
    mom = np.concatenate([inv.patch_view(data, int(o), p, 2, 4)[p // 2, 1:-1, 1] for o in offsets])
    return xc, depth, mom / depth


def check_dam_break_converges(update, fill, resolutions=(64, 128, 256, 512), t_end=0.04):
    """Under refinement the depth converges in L1 to Stoker's exact solution at a rate
    between 0.5 and 1.2 (a first-order scheme across a shock and a rarefaction), and the
    middle state's velocity approaches the exact um."""
    errs = []
    for cells in resolutions:
        x, d, u = dam_break(update, fill, cells, t_end=t_end)
        exact, hm, um = stoker_depth(x, t_end, 0.5, 2.0, 1.0)
        errs.append(np.sum(np.abs(d - exact)) / cells)
    rates = [np.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert all(0.5 <= r <= 1.2 for r in rates), (errs, rates)
    assert errs[-1] < 5.0 / resolutions[-1], errs   # 0.7 % at 512 cells, 1.2 % at 256
    # the plateau between rarefaction tail and shock carries the exact middle velocity
    xs = x[(x > 0.5 + 0.02) & (x < 0.5 + 0.08)]
    mid = u[(x > 0.5 + 0.02) & (x < 0.5 + 0.08)]
    assert len(xs) > 0 and np.max(np.abs(mid - um)) < 0.03 * um, (np.max(np.abs(mid - um)), um)
    return errs
