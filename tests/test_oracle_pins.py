"""The CPU oracle against what the mathematics fixes (no GPU needed).

Each property is defined in ``tests/invariants.py``; here it runs against the
oracle for every supported (dim, N).  None of these checks re-types the
oracle's formulas: they use exact invariants, a closed form for a special case,
an exact-arithmetic evaluation of a one-volume patch, and convergence to an
analytic solution of the linearised PDE.
"""
from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from tests import invariants as inv

CASES = [(2, 5), (2, 4), (3, 5)]


def oracle_step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic):
    return oracle.batch_update(data, sizes, offsets, dim, nq, dt, h, gamma, periodic)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.load()


@pytest.mark.parametrize("dim,nq", CASES)
def test_constant_state(dim, nq):
    inv.check_constant_state(oracle_step, dim, nq)


@pytest.mark.parametrize("dim,nq", CASES)
def test_conservation_periodic(dim, nq):
    inv.check_conservation(oracle_step, dim, nq)


@pytest.mark.parametrize("dim,nq", CASES)
def test_mirror_symmetry(dim, nq):
    inv.check_mirror(oracle_step, dim, nq)


@pytest.mark.parametrize("dim,nq", CASES)
def test_axis_permutation(dim, nq):
    inv.check_permutation(oracle_step, dim, nq)


def test_dimension_reduction():
    inv.check_dimension_reduction(oracle_step)


def test_passive_scalar_closed_form():
    inv.check_passive_scalar(oracle_step)
    inv.check_passive_scalar(oracle_step, u0=0.44, p0=1.21, seed=11)


@pytest.mark.parametrize("dim,nq", CASES)
def test_corner_halos_never_read(dim, nq):
    inv.check_corner_independence(oracle_step, dim, nq)


@pytest.mark.parametrize("dim,nq", CASES)
def test_lambda_reduction(dim, nq):
    inv.check_lambda_reduction(oracle_step, dim, nq)


@pytest.mark.parametrize("dim,nq", CASES)
def test_nan_propagates(dim, nq):
    inv.check_nan_propagates(oracle_step, dim, nq)


@pytest.mark.parametrize("mvec", [(1, 0), (1, 1)])
def test_acoustic_convergence_2d(mvec):
    errs, rates = inv.check_acoustic_convergence(oracle_step, 2, 5, mvec)
    # the error is a small multiple of h, far above rounding
    assert errs[-1] > 1e-4


def test_acoustic_convergence_2d_n4():
    inv.check_acoustic_convergence(oracle_step, 2, 4, (0, 1), sizes=(32, 64, 128))


@pytest.mark.slow
def test_acoustic_convergence_3d():
    # along z (the 3D-only axis); x and y are tied to z by the permutation check
    inv.check_acoustic_convergence(oracle_step, 3, 5, (0, 0, 1), sizes=(16, 32, 64))


# --------------------------------------------------------------------------- exact one-volume case
def _exact_step_one_volume(qs, dim, nq, gamma, dt, h):
    """Independent high-precision evaluation of one step of a p = 1 patch:
    the centre volume and its 2d face neighbours, with mpmath at 60 digits.
    qs: dict name -> state, names 'c', and ('lo', n) / ('hi', n)."""
    mpmath.mp.dps = 60
    g = mpmath.mpf(gamma)

    def terms(q, n):
        q = [mpmath.mpf(x) for x in q]
        rho, E = q[0], q[nq - 1]
        mom = q[1:nq - 1]
        pres = (g - 1) * (E - sum(m * m for m in mom) / (2 * rho))
        un = mom[n] / rho
        f = [mom[n]] + [mom[a] * un + (pres if a == n else 0) for a in range(len(mom))] + [(E + pres) * un]
        return f, abs(un) + mpmath.sqrt(g * pres / rho)

    def face(qL, qR, n):
        fL, lL = terms(qL, n)
        fR, lR = terms(qR, n)
        s = max(lL, lR)
        return [(fL[i] + fR[i]) / 2 - s * (mpmath.mpf(qR[i]) - mpmath.mpf(qL[i])) / 2 for i in range(nq)]

    r = mpmath.mpf(dt) / mpmath.mpf(h)
    D = [mpmath.mpf(0)] * nq
    for n in range(dim):
        left = face(qs[("lo", n)], qs["c"], n)
        right = face(qs["c"], qs[("hi", n)], n)
        D = [D[i] + left[i] - right[i] for i in range(nq)]
    new = [mpmath.mpf(qs["c"][i]) + r * D[i] for i in range(nq)]
    lam = max(terms(new, n)[1] for n in range(dim))
    return [float(x) for x in new], float(lam)


@pytest.mark.parametrize("dim,nq", CASES)
def test_one_volume_patch_high_precision(dim, nq):
    rng = np.random.Generator(np.random.PCG64(20 + dim + nq))
    p = 1
    n = p + 2
    vol = inv.primitives_to_state(rng.uniform(0.5, 1.5, n ** dim),
                                  [rng.uniform(-0.5, 0.5, n ** dim) for _ in range(3)],
                                  rng.uniform(0.5, 1.5, n ** dim), nq).reshape((n,) * dim + (nq,))
    data, sizes, offsets = inv.single_patch(p, dim, nq, vol)
    dt, h = 3.1e-3, 1.0 / 48.0
    out, lam = oracle.batch_update(data, sizes, offsets, dim, nq, dt, h, 1.4, False)
    centre = (1,) * dim
    qs = {"c": vol[centre]}
    for a in range(dim):
        ax = dim - 1 - a  # array axis of spatial axis a
        lo = list(centre)
        hi = list(centre)
        lo[ax] = 0
        hi[ax] = 2
        qs[("lo", a)] = vol[tuple(lo)]
        qs[("hi", a)] = vol[tuple(hi)]
    want, want_lam = _exact_step_one_volume(qs, dim, nq, 1.4, dt, h)
    got = out.reshape(vol.shape)[centre]
    scale = np.maximum(np.abs(want), 1.0)
    assert np.all(np.abs(got - want) <= 1e-14 * scale), (got, want)
    assert abs(lam[0] - want_lam) <= 4e-16 * want_lam


def test_rusanov_flux_of_equal_states_is_physical_flux():
    """Eq. 2 with Q+ == Q- collapses to F_n(Q) exactly (Fractions-free check)."""
    q = np.array([1.1, 0.2, -0.3, 0.05, 2.9])
    for n in range(3):
        f, _ = oracle.flux(q, n, 5)
        assert np.array_equal(oracle.rusanov(q, q, n, 5), f)


def test_euler_flux_rational_case():
    """F_n of a state with exactly representable primitives, checked in rational arithmetic."""
    rho, u, v, w, pres = Fraction(1, 2), Fraction(1, 4), Fraction(-1, 8), Fraction(1, 16), Fraction(3, 4)
    gamma = Fraction(7, 5)
    E = pres / (gamma - 1) + rho * (u * u + v * v + w * w) / 2
    q = np.array([float(rho), float(rho * u), float(rho * v), float(rho * w), float(E)])
    assert float(E) == E  # exactly representable
    vel = [u, v, w]
    for n in range(3):
        f, lam = oracle.flux(q, n, 5, 1.4)
        un = vel[n]
        want = [rho * un] + [rho * vel[a] * un + (pres if a == n else 0) for a in range(3)] + [(E + pres) * un]
        np.testing.assert_allclose(f, [float(x) for x in want], rtol=4e-16, atol=1e-17)
        assert abs(lam - (abs(float(un)) + math.sqrt(1.4 * 0.75 / 0.5))) <= 4e-16 * lam
