"""Run the HIP path through the C ABI from tests (numpy in, numpy out)."""
from __future__ import annotations

import numpy as np

from paper_2306_16731_amd import fvpatch as fv

DEVICE = "cuda:0"


def torch():
    import torch as _t
    return _t


def to_dev(a: np.ndarray):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(a)).to(DEVICE)


def gpu_step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic, *, pass_offsets=True):
    """One step through fv_patch_batch_update.  ``out`` starts as a copy of the input."""
    t = torch()
    d_in = to_dev(np.asarray(data, np.float64))
    d_out = d_in.clone()
    T = len(sizes)
    lam = t.full((T,), -1.0, dtype=t.float64, device=DEVICE)
    fv.fv_patch_batch_update(d_in, d_out, np.asarray(sizes, np.int32),
                             np.asarray(offsets, np.int64) if pass_offsets else None, T, dim, nq, dt, h, gamma,
                             fv.FV_HALO_PERIODIC if periodic else 0, lam)
    t.cuda.synchronize()
    return d_out.cpu().numpy(), lam.cpu().numpy()


def gpu_step_contiguous(data, sizes, offsets, dim, nq, dt, h, gamma, periodic):
    return gpu_step(data, sizes, offsets, dim, nq, dt, h, gamma, periodic, pass_offsets=False)


def gpu_run_steps(data, sizes, offsets, dim, nq, dts, h, gamma=1.4, periodic=False, pass_offsets=True):
    """len(dts) steps with device ping-pong buffers; returns (state, [lambda per step])."""
    t = torch()
    a = to_dev(np.asarray(data, np.float64))
    b = a.clone()
    T = len(sizes)
    lam = t.empty((len(dts), T), dtype=t.float64, device=DEVICE)
    sz = np.asarray(sizes, np.int32)
    of = np.asarray(offsets, np.int64) if pass_offsets else None
    for s, dt in enumerate(dts):
        fv.fv_patch_batch_update(a, b, sz, of, T, dim, nq, dt, h, gamma,
                                 fv.FV_HALO_PERIODIC if periodic else 0, lam[s])
        a, b = b, a
    t.cuda.synchronize()
    return a.cpu().numpy(), list(lam.cpu().numpy())


def component_errors(got: np.ndarray, want: np.ndarray, nq: int) -> np.ndarray:
    """Per-unknown max-norm error relative to the max-norm of the reference."""
    g = got.reshape(-1, nq)
    w = want.reshape(-1, nq)
    num = np.max(np.abs(g - w), axis=0)
    den = np.max(np.abs(w), axis=0)
    den = np.where(den > 0, den, np.max(np.abs(w)))
    return num / den


def lambda_error(got, want) -> float:
    got = np.asarray(got)
    want = np.asarray(want)
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
