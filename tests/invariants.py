"""Properties that any correct implementation of the Rusanov FV patch step has.

Every check takes a ``step`` callable

    step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic) -> (out, lam)

that applies ONE explicit Euler step to a flat batch (numpy float64 in, numpy
out; ``out`` starts as a copy of ``data`` so unwritten volumes keep their input
values) and returns the per-patch maximum wave speed of the new interior.  The
oracle and the HIP path are both run through these checks.

What each property pins (paper: conservative update of Sec. 2.2, Rusanov flux
Eq. 2, Euler user terms of Sec. 5, per-patch eigenvalue at the end of Sec. 2.2):
  * constant states are reproduced exactly: F_L == F_R and Q_R - Q_L == 0 on
    every face, whatever the flux is -- pins that only flux DIFFERENCES enter;
  * the eigenvalue of a constant state is max_n |u_n| + c computed from the
    primitives it was built from -- pins lambda_max,n = |u_n| + c;
  * discrete conservation on periodic patches -- pins that each face flux
    enters its two volumes with opposite signs;
  * mirror and axis-permutation symmetry -- pin that every axis is treated
    alike and that the sign conventions of the momenta are consistent;
  * reduction of a 3D patch that is uniform along y and z to the 2D patch --
    pins the 3D x-direction against 2D;
  * a one-step closed form for a passive scalar (textbook local
    Lax-Friedrichs for linear advection) -- pins the dissipation factor 1/2,
    the scaling dt/h and the sign of the update;
  * first-order convergence to the linearised acoustic plane wave -- pins the
    pressure terms, the energy flux and gamma;
  * corner / edge halo volumes never influence the result.
"""
from __future__ import annotations

import math

import numpy as np

from paper_2306_16731_amd import workloads as wl

GAMMA = 1.4
EPS = 2.0 ** -52


# ----------------------------------------------------------------------------- helpers
def patch_view(data: np.ndarray, off: int, p: int, dim: int, nq: int) -> np.ndarray:
    """Patch as an array indexed [k, j, i, q] (3D) or [j, i, q] (2D)."""
    n = (p + 2) ** dim * nq
    return data[off:off + n].reshape((p + 2,) * dim + (nq,))


def interior(view: np.ndarray, dim: int) -> np.ndarray:
    return view[(slice(1, -1),) * dim]


def face_halo_mask(p: int, dim: int) -> np.ndarray:
    """True for interior and face-halo volumes, False for corners / edges."""
    idx = np.indices((p + 2,) * dim)
    outside = sum(((a == 0) | (a == p + 1)).astype(int) for a in idx)
    return outside <= 1


def periodic_fill(view: np.ndarray, dim: int) -> None:
    """Self-wrap of every face halo of a single patch (numpy indexing, in place)."""
    p = view.shape[0] - 2
    for ax in range(dim):
        sl_lo = [slice(1, p + 1)] * dim
        sl_hi = [slice(1, p + 1)] * dim
        src_lo = [slice(1, p + 1)] * dim
        src_hi = [slice(1, p + 1)] * dim
        sl_lo[ax], src_lo[ax] = 0, p
        sl_hi[ax], src_hi[ax] = p + 1, 1
        view[tuple(sl_lo)] = view[tuple(src_lo)]
        view[tuple(sl_hi)] = view[tuple(src_hi)]


def primitives_to_state(rho, vel, pres, nq, gamma=GAMMA):
    """vel: list of velocity arrays (2 or 3 components)."""
    shape = np.shape(rho)
    flat = [np.asarray(x, float).reshape(-1) for x in (rho, *vel, pres)]
    rho_, u, v = flat[0], flat[1], flat[2]
    w = flat[3] if len(vel) > 2 else np.zeros_like(u)
    q = wl.conserved(rho_, u, v, w, flat[-1], nq, gamma)
    return q.reshape(tuple(shape) + (nq,))


def single_patch(p, dim, nq, vol_state):
    """Batch of one patch from volume states shaped [(p+2)]*dim + [nq]."""
    data = np.ascontiguousarray(vol_state, dtype=np.float64).reshape(-1).copy()
    return data, np.array([p], np.int32), np.array([0], np.int64)


def random_batch(rng, T, p, dim, nq):
    b = wl.make_batch(np.full(T, p, np.int32), dim, nq, rng=rng)
    return b.data, b.sizes, b.offsets


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


# ----------------------------------------------------------------------------- properties
def check_constant_state(step, dim, nq, p=5, T=3, seed=0, gamma=GAMMA):
    """Uniform Q per patch (interior + halo) is reproduced bitwise; lambda = max|u_n| + c."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vols = (p + 2) ** dim
    chunks, lam_expect = [], []
    for _ in range(T):
        rho = rng.uniform(0.5, 1.5)
        vel = [rng.uniform(-0.5, 0.5) for _ in range(3 if (dim == 3 or nq == 5) else 2)]
        pres = rng.uniform(0.5, 1.5)
        q = primitives_to_state([rho], [[x] for x in vel] + ([[0.0]] if len(vel) == 2 else []), [pres], nq, gamma)[0]
        chunks.append(np.tile(q, vols))
        c = math.sqrt(gamma * pres / rho)
        lam_expect.append(max(abs(x) for x in vel[:dim]) + c)
    data = np.concatenate(chunks)
    sizes = np.full(T, p, np.int32)
    offsets = np.arange(T, dtype=np.int64) * vols * nq
    dt, h = 0.37e-3, 1.0 / 48.0
    for periodic in (False, True):
        out, lam = step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic)
        assert np.array_equal(out, data), "constant state not reproduced bitwise"
        # c is built from primitives here and from conserved variables by the step:
        # agreement to a few ulps, not bitwise.
        np.testing.assert_allclose(lam, lam_expect, rtol=8 * EPS, atol=0)


def check_conservation(step, dim, nq, p=7, T=4, seed=1, gamma=GAMMA):
    """Periodic patches: the interior sum of every unknown is conserved up to rounding."""
    rng = np.random.Generator(np.random.PCG64(seed))
    data, sizes, offsets = random_batch(rng, T, p, dim, nq)
    for t in range(T):
        periodic_fill(patch_view(data, offsets[t], p, dim, nq), dim)
    h = 1.0 / 48.0
    dt = 0.4 * h / (dim * 3.0)
    out, _ = step(data, sizes, offsets, dim, nq, dt, h, gamma, True)
    r = dt / h
    for t in range(T):
        qi = interior(patch_view(data, offsets[t], p, dim, nq), dim).reshape(-1, nq)
        qo = interior(patch_view(out, offsets[t], p, dim, nq), dim).reshape(-1, nq)
        for q in range(nq):
            before = math.fsum(qi[:, q])
            after = math.fsum(qo[:, q])
            net = np.abs(qo[:, q] - qi[:, q])
            bound = 16 * EPS * math.fsum(np.abs(qi[:, q]) + net) + 16 * EPS * r
            assert abs(after - before) <= bound, (t, q, after - before, bound)
        # the periodic output halo is the self-wrap of the new interior
        v = patch_view(out, offsets[t], p, dim, nq).copy()
        w = v.copy()
        periodic_fill(w, dim)
        m = face_halo_mask(p, dim)
        assert np.array_equal(v[m], w[m])


def mirror(view: np.ndarray, axis_from_last: int, dim: int) -> np.ndarray:
    """Reflect a patch along axis n (0 = x) and negate the n-momentum."""
    ax = dim - 1 - axis_from_last
    m = np.flip(view, axis=ax).copy()
    m[..., 1 + axis_from_last] *= -1.0
    return m


def check_mirror(step, dim, nq, p=6, seed=2, gamma=GAMMA):
    """Reflection along every axis commutes with the step, bitwise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    data, sizes, offsets = random_batch(rng, 1, p, dim, nq)
    h, dt = 1.0 / 48.0, 1.1e-3
    out, lam = step(data, sizes, offsets, dim, nq, dt, h, gamma, False)
    vin = patch_view(data, 0, p, dim, nq)
    vout = patch_view(out, 0, p, dim, nq)
    for n in range(dim):
        mdata = mirror(vin, n, dim).reshape(-1).copy()
        mout, mlam = step(mdata, sizes, offsets, dim, nq, dt, h, gamma, False)
        got = interior(patch_view(mout, 0, p, dim, nq), dim)
        want = interior(mirror(vout, n, dim), dim)
        assert np.array_equal(got, want), f"mirror along axis {n} not bitwise"
        assert np.array_equal(mlam, lam)


def permute_axes(view: np.ndarray, a: int, b: int, dim: int) -> np.ndarray:
    """Swap spatial axes a and b (0 = x) and the matching momenta."""
    t = np.swapaxes(view, dim - 1 - a, dim - 1 - b).copy()
    t[..., [1 + a, 1 + b]] = t[..., [1 + b, 1 + a]]
    return t


def check_permutation(step, dim, nq, p=6, seed=3, gamma=GAMMA):
    """Swapping x and y (with m_x and m_y) commutes with the step, bitwise.
    In 3D the swaps involving z hold to rounding (the axis sums are ordered)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    data, sizes, offsets = random_batch(rng, 1, p, dim, nq)
    h, dt = 1.0 / 48.0, 1.1e-3
    out, lam = step(data, sizes, offsets, dim, nq, dt, h, gamma, False)
    vin = patch_view(data, 0, p, dim, nq)
    vout = patch_view(out, 0, p, dim, nq)
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
    for a, b in pairs:
        pdata = permute_axes(vin, a, b, dim).reshape(-1).copy()
        pout, plam = step(pdata, sizes, offsets, dim, nq, dt, h, gamma, False)
        got = interior(patch_view(pout, 0, p, dim, nq), dim)
        want = interior(permute_axes(vout, a, b, dim), dim)
        if (a, b) == (0, 1):
            assert np.array_equal(got, want), f"swap {a}<->{b} not bitwise"
        else:
            assert rel_err(got, want) <= 64 * EPS
        np.testing.assert_allclose(plam, lam, rtol=4 * EPS, atol=0)


def check_dimension_reduction(step, p=6, seed=4, gamma=GAMMA):
    """A 3D patch uniform along y and z gives, bitwise, the 2D (N=5) patch uniform along y."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = p + 2
    rho = rng.uniform(0.5, 1.5, n)
    u, v, w = (rng.uniform(-0.5, 0.5, n) for _ in range(3))
    pres = rng.uniform(0.5, 1.5, n)
    line = primitives_to_state(rho, [u, v, w], pres, 5, gamma)  # [n, 5]
    v2 = np.broadcast_to(line, (n, n, 5)).copy()
    v3 = np.broadcast_to(line, (n, n, n, 5)).copy()
    h, dt = 1.0 / 48.0, 1.3e-3
    d2, s2, o2 = single_patch(p, 2, 5, v2)
    d3, s3, o3 = single_patch(p, 3, 5, v3)
    out2, lam2 = step(d2, s2, o2, 2, 5, dt, h, gamma, False)
    out3, lam3 = step(d3, s3, o3, 3, 5, dt, h, gamma, False)
    i2 = interior(patch_view(out2, 0, p, 2, 5), 2)
    i3 = interior(patch_view(out3, 0, p, 3, 5), 3)
    for k in range(p):
        assert np.array_equal(i3[k], i2), "3D patch uniform in y,z differs from 2D"
    # the 3D eigenvalue also sees |w| + c, the 2D one only |u|, |v|
    assert lam3[0] >= lam2[0]


def check_passive_scalar(step, p=9, seed=5, gamma=GAMMA, u0=-0.31, p0=0.83):
    """2D, N = 5: rho = 1, u = u0, v = 0, p = p0 uniform, arbitrary m_z.
    One step is textbook local Lax-Friedrichs for linear advection of m_z and E:
      q_new = q - r [ u0/2 (q_{i+1} - q_{i-1}) - lx/2 (q_{i+1} - 2q + q_{i-1})
                                               - ly/2 (q_{j+1} - 2q + q_{j-1}) ]
    with lx = |u0| + c0, ly = c0, c0 = sqrt(gamma p0), r = dt / h;
    rho, m_x, m_y are unchanged up to rounding."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = p + 2
    mz = rng.uniform(-0.5, 0.5, (n, n))
    ones = np.ones((n, n))
    vol = primitives_to_state(ones, [u0 * ones, 0.0 * ones, mz], p0 * ones, 5, gamma).reshape(n, n, 5)
    data, sizes, offsets = single_patch(p, 2, 5, vol)
    h, dt = 1.0 / 48.0, 2.2e-3
    r = dt / h
    out, _ = step(data, sizes, offsets, 2, 5, dt, h, gamma, False)
    got = interior(patch_view(out, 0, p, 2, 5), 2)
    c0 = math.sqrt(gamma * p0)
    lx, ly = abs(u0) + c0, c0
    for q in (3, 4):
        f = vol[..., q]
        c = f[1:-1, 1:-1]
        xp, xm = f[1:-1, 2:], f[1:-1, :-2]
        yp, ym = f[2:, 1:-1], f[:-2, 1:-1]
        want = c - r * (0.5 * u0 * (xp - xm) - 0.5 * lx * (xp - 2 * c + xm) - 0.5 * ly * (yp - 2 * c + ym))
        assert rel_err(got[..., q], want) <= 1e-14, (q, rel_err(got[..., q], want))
    for q in (0, 1, 2):
        assert np.max(np.abs(got[..., q] - vol[1:-1, 1:-1, q])) <= 1e-14


def acoustic_error(step, p, dim, nq, mvec, eps=1e-6, t_end=0.25, gamma=GAMMA):
    """Max-norm error (relative to the amplitude) against the linearised acoustic
    plane wave on one periodic patch covering [0,1]^d with h = 1/p.
      rho = 1 + eps sin(phi), u = eps m/|m| sin(phi), p = 1/gamma + eps sin(phi),
      phi = 2 pi m.x - omega t, omega = 2 pi |m|  (c0 = 1)."""
    h = 1.0 / p
    mvec = np.asarray(mvec, float)
    mn = float(np.linalg.norm(mvec))
    khat = mvec / mn
    omega = 2 * math.pi * mn
    centres = (np.arange(p + 2) - 0.5) * h
    grids = np.meshgrid(*([centres] * dim), indexing="ij")  # grids[a] is the coordinate a, array [x,y(,z)]

    def state(t):
        phi = 2 * math.pi * sum(mvec[a] * grids[a] for a in range(dim)) - omega * t
        s = np.sin(phi)
        rho = 1.0 + eps * s
        vel = [eps * khat[a] * s for a in range(dim)] + ([np.zeros_like(s)] if (nq == 5 and dim == 2) else [])
        st = primitives_to_state(rho.reshape(-1), [x.reshape(-1) for x in vel], (1.0 / gamma + eps * s).reshape(-1), nq, gamma)
        st = st.reshape(s.shape + (nq,))
        # meshgrid is (x, y, z) indexed; patch layout is (z, y, x)
        return np.ascontiguousarray(np.transpose(st, tuple(range(dim))[::-1] + (dim,)))

    nsteps = int(math.ceil(t_end / (0.4 * h / (dim * (1 + 2 * eps)))))
    dt = t_end / nsteps
    data, sizes, offsets = single_patch(p, dim, nq, state(0.0))
    for _ in range(nsteps):
        data, _ = step(data, sizes, offsets, dim, nq, dt, h, gamma, True)
    got = interior(patch_view(data, 0, p, dim, nq), dim)
    want = interior(state(t_end), dim)
    return float(np.max(np.abs(got - want))) / eps


def check_acoustic_convergence(step, dim, nq, mvec, sizes=(16, 32, 64, 128)):
    errs = [acoustic_error(step, p, dim, nq, mvec) for p in sizes]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    for r in rates[-2:]:
        assert 0.8 <= r <= 1.2, (errs, rates)
    return errs, rates


def check_corner_independence(step, dim, nq, p=5, T=3, seed=6, gamma=GAMMA):
    """NaN in corner / edge halo volumes changes nothing (they are never read)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    data, sizes, offsets = random_batch(rng, T, p, dim, nq)
    poisoned = data.copy()
    mask = ~face_halo_mask(p, dim)
    for t in range(T):
        v = patch_view(poisoned, offsets[t], p, dim, nq)
        v[mask] = np.nan
    h, dt = 1.0 / 48.0, 1e-3
    for periodic in (False, True):
        out, lam = step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic)
        pout, plam = step(poisoned, sizes, offsets, dim, nq, dt, h, gamma, periodic)
        for t in range(T):
            a = patch_view(out, offsets[t], p, dim, nq)[face_halo_mask(p, dim)]
            b = patch_view(pout, offsets[t], p, dim, nq)[face_halo_mask(p, dim)]
            assert np.all(np.isfinite(b)) and np.array_equal(a, b)
        assert np.array_equal(lam, plam)


def independent_lambda(out, sizes, offsets, dim, nq, gamma=GAMMA):
    """max over interior volumes and axes of |u_n| + c, straight from numpy."""
    res = []
    for t in range(len(sizes)):
        q = interior(patch_view(out, offsets[t], int(sizes[t]), dim, nq), dim).reshape(-1, nq)
        rho = q[:, 0]
        mom = q[:, 1:nq - 1]
        pres = (gamma - 1.0) * (q[:, nq - 1] - 0.5 * np.sum(mom * mom, axis=1) / rho)
        c = np.sqrt(gamma * pres / rho)
        res.append(np.max(np.abs(mom[:, :dim]) / rho[:, None] + c[:, None]))
    return np.array(res)


def check_lambda_reduction(step, dim, nq, p=7, T=5, seed=7, gamma=GAMMA):
    rng = np.random.Generator(np.random.PCG64(seed))
    data, sizes, offsets = random_batch(rng, T, p, dim, nq)
    out, lam = step(data, sizes, offsets, dim, nq, 1e-3, 1.0 / 48.0, gamma, False)
    np.testing.assert_allclose(lam, independent_lambda(out, sizes, offsets, dim, nq, gamma), rtol=8 * EPS, atol=0)


def check_nan_propagates(step, dim, nq, p=4, seed=8, gamma=GAMMA):
    """A negative pressure in one interior volume yields a NaN eigenvalue for its patch only."""
    rng = np.random.Generator(np.random.PCG64(seed))
    data, sizes, offsets = random_batch(rng, 3, p, dim, nq)
    v = patch_view(data, offsets[1], p, dim, nq)
    centre = (p // 2 + 1,) * dim
    v[centre + (nq - 1,)] = -10.0  # E < kinetic energy -> p < 0 -> c = NaN
    out, lam = step(data, sizes, offsets, dim, nq, 1e-4, 1.0 / 48.0, gamma, False)
    assert np.isnan(lam[1]) and np.isfinite(lam[0]) and np.isfinite(lam[2])
