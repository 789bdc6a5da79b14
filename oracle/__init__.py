"""Plain FP64 CPU oracle for the Rusanov Finite Volume patch update.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check and to time the GPU path.  The product
library never imports it, and it imports nothing from the product package.

The arithmetic lives in ``fv_oracle.c`` (plain C, compiled with
``-O2 -ffp-contract=off``, no fast-math); this module only builds it with gcc
and marshals numpy arrays through ctypes.  Every function follows the paper's
definitions: the conservative update (Sec. 2.2), the Rusanov flux (Eq. 2), the
Euler user terms F_n / lambda_max,n (Sec. 5, Eq. 1 with B = S = delta = 0) and
the per-patch eigenvalue reduction for the CFL condition (end of Sec. 2.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "fv_oracle.c")
LIBRARY = os.path.join(_HERE, "libfvoracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(source: str = SOURCE, output: str = LIBRARY, extra: list[str] | None = None) -> str:
    """Compile the oracle with gcc.  Returns the path of the shared library."""
    cmd = ["gcc", *CFLAGS, *(extra or []), "-o", output, source, "-lm"]
    subprocess.run(cmd, check=True)
    return output


_lib = None


def load(path: str | None = None, rebuild: bool = False):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None or rebuild:
        if rebuild or not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
            build()
        _lib = _bind(ctypes.CDLL(LIBRARY))
    return _lib


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    i32, f64 = ctypes.c_int32, ctypes.c_double
    lib.fvo_batch_update.argtypes = [dp, dp, ip, lp, i32, i32, i32, f64, f64, f64, i32, dp, i32]
    lib.fvo_batch_update.restype = ctypes.c_int
    lib.fvo_batch_lambda.argtypes = [dp, ip, lp, i32, i32, i32, f64, dp]
    lib.fvo_batch_lambda.restype = ctypes.c_int
    lib.fvo_batch_wrap.argtypes = [dp, ip, lp, i32, i32, i32]
    lib.fvo_batch_wrap.restype = ctypes.c_int
    lib.fvo_flux.argtypes = [dp, i32, i32, f64, dp, dp]
    lib.fvo_flux.restype = None
    lib.fvo_rusanov.argtypes = [dp, dp, i32, i32, f64, dp]
    lib.fvo_rusanov.restype = None
    lib.fvo_max_threads.argtypes = []
    lib.fvo_max_threads.restype = ctypes.c_int32
    lib.fvo_halo_fill.argtypes = [dp, dp, ip, lp, ip, i32, i32, i32]
    lib.fvo_halo_fill.restype = ctypes.c_int
    lib.fvo_batch_update_lts.argtypes = [dp, dp, ip, lp, i32, i32, i32, dp, dp, f64, dp, i32]
    lib.fvo_batch_update_lts.restype = ctypes.c_int
    lib.fvo_local_dt.argtypes = [dp, dp, i32, i32, f64, dp]
    lib.fvo_local_dt.restype = ctypes.c_int
    lib.fvo_pde_shape.argtypes = [i32, i32, ip, ip, ip]
    lib.fvo_pde_shape.restype = ctypes.c_int
    lib.fvo_pde_update.argtypes = [i32, dp, i32, dp, dp, ip, lp, i32, i32, f64, f64, i32, dp]
    lib.fvo_pde_update.restype = ctypes.c_int
    lib.fvo_pde_terms.argtypes = [i32, i32, dp, dp, i32, dp, dp, dp, dp, dp]
    lib.fvo_pde_terms.restype = ctypes.c_int
    return lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _descriptors(sizes, offsets, num_patches):
    sizes = np.ascontiguousarray(np.broadcast_to(np.asarray(sizes, dtype=np.int32), (num_patches,)))
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    assert offsets.shape == (num_patches,)
    return sizes, offsets


def batch_update(state_in: np.ndarray, sizes, offsets, dim: int, nq: int, dt: float, h: float,
                 gamma: float = 1.4, periodic: bool = False, out: np.ndarray | None = None,
                 want_lambda: bool = True, nthreads: int = 0, lib=None):
    """One explicit Euler step of every patch.  Returns (out, lambda or None).

    ``out`` defaults to a copy of ``state_in`` so that volumes the step does not
    write (halos, corners) keep their input values.
    """
    lib = lib or load()
    num_patches = len(offsets)
    sizes, offsets = _descriptors(sizes, offsets, num_patches)
    state_in = np.ascontiguousarray(state_in, dtype=np.float64)
    if out is None:
        out = state_in.copy()
    lam = np.zeros(num_patches, dtype=np.float64) if want_lambda else None
    rc = lib.fvo_batch_update(_dptr(state_in), _dptr(out),
                              sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              num_patches, dim, nq, dt, h, gamma, int(bool(periodic)),
                              _dptr(lam) if lam is not None else None, nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out, lam


def batch_lambda(state: np.ndarray, sizes, offsets, dim: int, nq: int, gamma: float = 1.4, lib=None):
    """Maximum wave speed over the interior of every patch of ``state``."""
    lib = lib or load()
    num_patches = len(offsets)
    sizes, offsets = _descriptors(sizes, offsets, num_patches)
    state = np.ascontiguousarray(state, dtype=np.float64)
    lam = np.zeros(num_patches, dtype=np.float64)
    rc = lib.fvo_batch_lambda(_dptr(state), sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              num_patches, dim, nq, gamma, _dptr(lam))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return lam


def batch_wrap(state: np.ndarray, sizes, offsets, dim: int, nq: int, lib=None) -> np.ndarray:
    """Periodic self-wrap of every patch's face halo, in place; returns ``state``."""
    lib = lib or load()
    num_patches = len(offsets)
    sizes, offsets = _descriptors(sizes, offsets, num_patches)
    rc = lib.fvo_batch_wrap(_dptr(state), sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), num_patches, dim, nq)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return state


def halo_fill(src: np.ndarray, sizes, offsets, neighbors, dim: int, nq: int, dst: np.ndarray | None = None,
              lib=None) -> np.ndarray:
    """Face halos of every patch from its neighbours (neighbors: [T, 2*dim], -1 = none).
    Writes into ``dst`` (default: a copy of ``src``) and returns it."""
    lib = lib or load()
    num_patches = len(offsets)
    sizes, offsets = _descriptors(sizes, offsets, num_patches)
    src = np.ascontiguousarray(src, dtype=np.float64)
    dst = src.copy() if dst is None else dst
    nb = np.ascontiguousarray(np.asarray(neighbors, dtype=np.int32).reshape(num_patches, 2 * dim))
    rc = lib.fvo_halo_fill(_dptr(src), _dptr(dst), sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), num_patches, dim, nq)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return dst


def batch_update_lts(state_in: np.ndarray, sizes, offsets, dim: int, nq: int, dt, h, gamma: float = 1.4,
                     out: np.ndarray | None = None, nthreads: int = 0, lib=None):
    """One step of every patch t with its own dt[t] and h[t].  Returns (out, lambda)."""
    lib = lib or load()
    num_patches = len(offsets)
    sizes, offsets = _descriptors(sizes, offsets, num_patches)
    state_in = np.ascontiguousarray(state_in, dtype=np.float64)
    out = state_in.copy() if out is None else out
    dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (num_patches,)))
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (num_patches,)))
    lam = np.zeros(num_patches, dtype=np.float64)
    rc = lib.fvo_batch_update_lts(_dptr(state_in), _dptr(out), sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), num_patches, dim, nq,
                                  _dptr(dt), _dptr(h), gamma, _dptr(lam), nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out, lam


def local_dt(lam, h, dim: int, cfl: float, lib=None) -> np.ndarray:
    """Per-patch step size cfl * h[t] / (dim * lambda[t])."""
    lib = lib or load()
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), lam.shape))
    out = np.zeros_like(lam)
    rc = lib.fvo_local_dt(_dptr(lam), _dptr(h), len(lam), dim, cfl, _dptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def flux(q, n: int, nq: int, gamma: float = 1.4, lib=None):
    """F_n(Q) and lambda_max,n(Q) of one volume."""
    lib = lib or load()
    q = np.ascontiguousarray(q, dtype=np.float64)
    f = np.zeros(nq)
    lam = ctypes.c_double()
    lib.fvo_flux(_dptr(q), n, nq, gamma, _dptr(f), ctypes.byref(lam))
    return f, lam.value


def rusanov(qL, qR, n: int, nq: int, gamma: float = 1.4, lib=None):
    """Rusanov flux through one face."""
    lib = lib or load()
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    f = np.zeros(nq)
    lib.fvo_rusanov(_dptr(qL), _dptr(qR), n, nq, gamma, _dptr(f))
    return f


def max_threads(lib=None) -> int:
    lib = lib or load()
    return int(lib.fvo_max_threads())


def run_steps(state: np.ndarray, sizes, offsets, dim: int, nq: int, dts, h: float, gamma: float = 1.4,
              periodic: bool = False, nthreads: int = 0):
    """Apply len(dts) steps with ping-pong buffers.  Returns (state, [lambda per step])."""
    a = np.ascontiguousarray(state, dtype=np.float64).copy()
    b = a.copy()
    lams = []
    for dt in dts:
        b, lam = batch_update(a, sizes, offsets, dim, nq, dt, h, gamma, periodic, out=b, nthreads=nthreads)
        lams.append(lam)
        a, b = b, a
    return a, lams


# ---------------------------------------------------------------- the generic solver of Eq. 1
PDE_EULER = 0
PDE_SHALLOW_WATER = 1
PDE_ADVECTION = 2
PDE_ACOUSTICS = 3
PDE_ACOUSTICS_NCP = 4


def pde_shape(pde: int, dim: int, lib=None) -> tuple[int, int, int]:
    """(unknowns per volume, evolved unknowns, parameters) of a PDE in dim dimensions."""
    lib = lib or load()
    nq, nv, npr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    if lib.fvo_pde_shape(pde, dim, ctypes.byref(nq), ctypes.byref(nv), ctypes.byref(npr)) != 0:
        raise ValueError(f"no PDE {pde} in {dim}D")
    return nq.value, nv.value, npr.value


def pde_update(pde: int, prm, state_in: np.ndarray, sizes, offsets, dim: int, dt: float, h: float,
               periodic: bool = False, out: np.ndarray | None = None, want_lambda: bool = True, lib=None):
    """One explicit Euler step of every patch for the PDE `pde` with parameters prm.
    Returns (out, lambda or None); ``out`` defaults to a copy of the input."""
    lib = lib or load()
    num_patches = len(offsets)
    sizes, offsets = _descriptors(sizes, offsets, num_patches)
    state_in = np.ascontiguousarray(state_in, dtype=np.float64)
    prm = np.ascontiguousarray(np.asarray(prm, np.float64).reshape(-1))
    out = state_in.copy() if out is None else out
    lam = np.zeros(num_patches, dtype=np.float64) if want_lambda else None
    rc = lib.fvo_pde_update(pde, _dptr(prm), len(prm), _dptr(state_in), _dptr(out),
                            sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), num_patches, dim, dt, h,
                            int(bool(periodic)), _dptr(lam) if lam is not None else None)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out, lam


def pde_terms(pde: int, dim: int, prm, q, n: int, dq=None, lib=None):
    """User terms of one volume: (F_n(q), lambda_max,n(q), B_n(q) dq, S(q)); vectors over
    the evolved unknowns."""
    lib = lib or load()
    nq, nv, _ = pde_shape(pde, dim, lib)
    prm = np.ascontiguousarray(np.asarray(prm, np.float64).reshape(-1))
    q = np.ascontiguousarray(np.asarray(q, np.float64))
    dq = np.zeros(nq) if dq is None else np.ascontiguousarray(np.asarray(dq, np.float64))
    f, b, s = np.zeros(nv), np.zeros(nv), np.zeros(nv)
    lam = np.zeros(1)
    if lib.fvo_pde_terms(pde, dim, _dptr(prm), _dptr(q), n, _dptr(dq), _dptr(f), _dptr(lam), _dptr(b),
                         _dptr(s)) != 0:
        raise ValueError("oracle rejected the arguments")
    return f, float(lam[0]), b, s
