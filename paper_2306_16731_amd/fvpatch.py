"""Python binding of the C ABI in include/fvpatch.h (ctypes; argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
buffers are passed as torch tensors on the GPU (float64, contiguous) or as raw
integer device addresses; host descriptor arrays as numpy arrays or
sequences.  The compute runs in the HIP library ``libfvpatch.so``; there is no
other implementation behind these names -- if the library is missing, loading
fails with an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # torch first: its HIP runtime is then the one the library binds to
    import torch
except ImportError:  # pragma: no cover - torch is part of the supported environment
    torch = None

LIBRARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfvpatch.so")

FV_OK = 0
FV_ERR_INVALID_ARG = -1
FV_ERR_UNSUPPORTED = -2
FV_ERR_NO_DEVICE = -3
FV_ERR_LAUNCH = -4
FV_ERR_OOM = -5
FV_ERR_BUDGET = -6
FV_ERR_OVERLAP = -7
FV_HALO_PERIODIC = 0x2
FV_MAX_P_2D = 64
FV_MAX_P_3D = 24
FV_MAX_OFFSET = 1 << 48
FV_NOALLOC_MAX_PATCHES = 262144

# Every symbol the header declares (checked by the tests against include/fvpatch.h).
EXPORTS = ["fv_patch_batch_update", "fv_patch_batch_update_noalloc", "fv_set_tuning", "fv_get_tuning", "fv_plan_create", "fv_plan_execute",
           "fv_plan_capture_steps", "fv_plan_replay", "fv_plan_info", "fv_plan_destroy", "fv_plan_get_tuning",
           "fv_server_create",
           "fv_server_add_mesh", "fv_server_submit", "fv_server_poll", "fv_server_drain", "fv_server_run_trace",
           "fv_server_read_mesh", "fv_server_stats_get", "fv_server_destroy", "fv_server_inject",
           "fv_server_batch_log", "fv_mesh_create",
           "fv_mesh_halo_fill", "fv_mesh_step", "fv_local_dt", "fv_mesh_destroy", "fv_flavour_update",
           "fv_host_patches_update", "fv_host_alloc", "fv_host_free", "fv_pde_unknowns", "fv_pde_batch_update", "fv_status_string",
           "fv_last_error", "fv_version", "fv_build_id"]
FV_SERVE_FUSED = 0
FV_SERVE_PLAIN = 1
FV_INJECT_FAIL = 1
FV_INJECT_HANG = 2
FV_HALO_FROM_IN = 0x4
FV_PLAN_NO_PERSIST = 0x100
FV_PLAN_PER_CLASS = 0x200
FV_KERNEL_AUTO = 0
FV_KERNEL_BLOCK = 1
FV_KERNEL_WAVE = 2
FV_KERNEL_TILE = 3
FV_KERNEL_FIXED = 4
FV_FLAVOUR_BATCHED = 1
FV_FLAVOUR_PATCH_WISE = 2
FV_FLAVOUR_TASK_GRAPH = 3
FV_PDE_EULER = 0
FV_PDE_SHALLOW_WATER = 1
FV_PDE_ADVECTION = 2
FV_PDE_ACOUSTICS = 3
FV_PDE_ACOUSTICS_NCP = 4
PDE_IDS = {"euler": FV_PDE_EULER, "shallow_water": FV_PDE_SHALLOW_WATER, "advection": FV_PDE_ADVECTION,
           "acoustics": FV_PDE_ACOUSTICS, "acoustics_ncp": FV_PDE_ACOUSTICS_NCP}
FV_TRANSFER_PIPELINED = 0
FV_TRANSFER_PER_PATCH = 1
FV_TRANSFER_STAGED = 2
FV_TRANSFER_ZERO_COPY = 3
FV_TRANSFER_MAX_SLOTS = 8
FV_TRANSFER_MAX_THREADS = 64
FIXED_SIZES_2D = (3, 5, 9, 16, 17)  # patch sizes with a fixed-size build (2D, unknowns = 5)
FIXED_SIZES_3D = (4, 6, 8)          # the same in 3D


class fv_tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("block", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("rows", ctypes.c_int32)]

    def as_dict(self):
        return {"kernel": self.kernel, "block": self.block, "prefetch": self.prefetch, "rows": self.rows}


class FvError(RuntimeError):
    """A non-zero fv_status returned by the library."""

    def __init__(self, status: int, detail: str):
        super().__init__(f"{status_name(status)} ({status}): {detail}")
        self.status = status
        self.detail = detail


class fv_plan_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("num_patches", "num_tasks", "num_class_launches", "prefetch",
                                                "lds_per_wave_bytes", "persistent", "captured_steps")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class fv_server_config(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("gamma", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("mode", ctypes.c_int32), ("max_inflight", ctypes.c_int32), ("max_retries", ctypes.c_int32),
                ("deadline_ms", ctypes.c_double)]


class fv_serve_request(ctypes.Structure):
    _fields_ = [("arrival_ns", ctypes.c_int64), ("mesh", ctypes.c_int32), ("first", ctypes.c_int32),
                ("count", ctypes.c_int32), ("reserved", ctypes.c_int32), ("dt", ctypes.c_double)]


SERVE_REQUEST_DTYPE = np.dtype([("arrival_ns", "<i8"), ("mesh", "<i4"), ("first", "<i4"), ("count", "<i4"),
                                ("reserved", "<i4"), ("dt", "<f8")])


class fv_server_stats(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int64) for n in ("submitted", "completed", "queued", "inflight", "peak_queued",
                                               "peak_inflight", "cells_updated", "failed", "retried",
                                               "resident_bytes", "budget_bytes")]
                + [(n, ctypes.c_double) for n in ("p50_ms", "p99_ms", "max_ms", "mean_ms", "cell_updates_per_s")])

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


BATCH_RECORD_DTYPE = np.dtype([("ticket", "<i8"), ("arrival_ns", "<i8"), ("launch_ns", "<i8"), ("done_ns", "<i8"),
                               ("cells", "<i8"), ("mesh", "<i4"), ("count", "<i4"), ("retries", "<i4"),
                               ("reserved", "<i4")])


class fv_transfer_config(ctypes.Structure):
    _fields_ = [("chunk_bytes", ctypes.c_int64), ("slots", ctypes.c_int32), ("host_threads", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class fv_transfer_stats(ctypes.Structure):
    _fields_ = [("bytes_to_device", ctypes.c_int64), ("bytes_to_host", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("host_copy_seconds", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def load(path: str = LIBRARY):
    """Load libfvpatch.so (built by ``python -m paper_2306_16731_amd.build``).  A library built from
    other sources than the ones beside it (its fv_build_id() differs from the hash of the current
    sources) is refused with ImportError, unless FVPATCH_ALLOW_STALE=1."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2306_16731_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    lib.fv_build_id.argtypes = []
    lib.fv_build_id.restype = ctypes.c_char_p
    if path == LIBRARY and os.environ.get("FVPATCH_ALLOW_STALE") != "1":
        from . import build as _build
        built, now = lib.fv_build_id().decode(), _build.source_hash()
        if built != now:
            raise ImportError(f"{path} was built from other sources (build id {built}, sources {now}): rebuild "
                              "it with `python -m paper_2306_16731_amd.build`")
    vp, i32, i64, f64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    lib.fv_patch_batch_update.argtypes = [vp, vp, vp, vp, i32, i32, i32, f64, f64, f64, u32, vp, vp]
    lib.fv_patch_batch_update.restype = ctypes.c_int
    lib.fv_patch_batch_update_noalloc.argtypes = [vp, vp, vp, vp, i32, i32, i32, f64, f64, f64, u32, vp, vp]
    lib.fv_patch_batch_update_noalloc.restype = ctypes.c_int
    lib.fv_status_string.argtypes = [ctypes.c_int]
    lib.fv_status_string.restype = ctypes.c_char_p
    lib.fv_last_error.argtypes = []
    lib.fv_last_error.restype = ctypes.c_char_p
    lib.fv_version.argtypes = []
    lib.fv_version.restype = i32
    lib.fv_set_tuning.argtypes = [i32, i32, i32, ctypes.POINTER(fv_tuning)]
    lib.fv_set_tuning.restype = ctypes.c_int
    lib.fv_get_tuning.argtypes = [i32, i32, i32, ctypes.POINTER(fv_tuning)]
    lib.fv_get_tuning.restype = ctypes.c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.fv_plan_create.argtypes = [pp, vp, vp, i32, i32, i32, u32, vp, i32]
    lib.fv_plan_create.restype = ctypes.c_int
    lib.fv_plan_get_tuning.argtypes = [vp, i32, ctypes.POINTER(fv_tuning)]
    lib.fv_plan_get_tuning.restype = ctypes.c_int
    lib.fv_plan_execute.argtypes = [vp, vp, vp, f64, vp, f64, f64, vp, vp]
    lib.fv_plan_execute.restype = ctypes.c_int
    lib.fv_plan_capture_steps.argtypes = [vp, i32, vp, vp, f64, f64, f64, vp, vp, vp]
    lib.fv_plan_capture_steps.restype = ctypes.c_int
    lib.fv_plan_replay.argtypes = [vp, vp]
    lib.fv_plan_replay.restype = ctypes.c_int
    lib.fv_plan_info.argtypes = [vp, ctypes.POINTER(fv_plan_stats)]
    lib.fv_plan_info.restype = ctypes.c_int
    lib.fv_plan_destroy.argtypes = [vp]
    lib.fv_plan_destroy.restype = ctypes.c_int
    sp = ctypes.POINTER(fv_server_stats)
    lib.fv_server_create.argtypes = [pp, ctypes.POINTER(fv_server_config)]
    lib.fv_server_add_mesh.argtypes = [vp, i32, i32, f64, vp, i32, vp, ctypes.POINTER(ctypes.c_int32)]
    lib.fv_server_inject.argtypes = [vp, i64, i32, i32]
    lib.fv_server_batch_log.argtypes = [vp, vp, i64, ctypes.POINTER(ctypes.c_int64)]
    lib.fv_server_submit.argtypes = [vp, i32, i32, i32, f64, i64, ctypes.POINTER(ctypes.c_int64)]
    lib.fv_server_poll.argtypes = [vp, sp]
    lib.fv_server_drain.argtypes = [vp, sp]
    lib.fv_server_run_trace.argtypes = [vp, vp, i64, sp]
    lib.fv_server_read_mesh.argtypes = [vp, i32, vp]
    lib.fv_server_stats_get.argtypes = [vp, sp]
    lib.fv_server_destroy.argtypes = [vp]
    for name in ("fv_server_create", "fv_server_add_mesh", "fv_server_submit", "fv_server_poll", "fv_server_drain",
                 "fv_server_inject", "fv_server_batch_log",
                 "fv_server_run_trace", "fv_server_read_mesh", "fv_server_stats_get", "fv_server_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    lib.fv_mesh_create.argtypes = [pp, vp, vp, vp, i32, i32, i32]
    lib.fv_mesh_halo_fill.argtypes = [vp, vp, vp]
    lib.fv_mesh_step.argtypes = [vp, vp, vp, vp, vp, f64, vp, vp]
    lib.fv_local_dt.argtypes = [vp, vp, i32, i32, f64, vp, vp]
    lib.fv_mesh_destroy.argtypes = [vp]
    for name in ("fv_mesh_create", "fv_mesh_halo_fill", "fv_mesh_step", "fv_local_dt", "fv_mesh_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    lib.fv_flavour_update.argtypes = [i32, vp, vp, vp, vp, i32, i32, i32, f64, f64, f64, u32, vp, vp]
    lib.fv_flavour_update.restype = ctypes.c_int
    lib.fv_host_patches_update.argtypes = [vp, vp, vp, i32, i32, i32, f64, f64, f64, u32, vp,
                                           ctypes.POINTER(fv_transfer_config), ctypes.POINTER(fv_transfer_stats)]
    lib.fv_host_patches_update.restype = ctypes.c_int
    lib.fv_host_alloc.argtypes = [ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
    lib.fv_host_alloc.restype = ctypes.c_int
    lib.fv_host_free.argtypes = [vp]
    lib.fv_host_free.restype = ctypes.c_int
    lib.fv_pde_unknowns.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.fv_pde_unknowns.restype = ctypes.c_int
    lib.fv_pde_batch_update.argtypes = [i32, vp, i32, vp, vp, vp, vp, i32, i32, f64, f64, u32, vp, vp]
    lib.fv_pde_batch_update.restype = ctypes.c_int
    _lib = lib
    return lib


def _dev_ptr(x):
    """Device address of a tensor (checked: on GPU, float64/int, contiguous) or a raw int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if torch is not None and isinstance(x, torch.Tensor):
        if not x.is_cuda:
            raise ValueError("device buffer must be a GPU tensor")
        if not x.is_contiguous():
            raise ValueError("device buffer must be contiguous")
        return x.data_ptr()
    raise TypeError(f"expected a GPU tensor or an int address, got {type(x)!r}")


def _host_array(x, dtype):
    if x is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(x, dtype=dtype))
    return a, a.ctypes.data


def _stream_handle(stream):
    if stream is None:
        if torch is not None and torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def status_name(status: int) -> str:
    return load().fv_status_string(int(status)).decode()


def fv_status_string(status: int) -> str:
    return load().fv_status_string(int(status)).decode()


def fv_last_error() -> str:
    return load().fv_last_error().decode()


def fv_version() -> int:
    return int(load().fv_version())


def _check(status: int) -> int:
    if status != FV_OK:
        raise FvError(status, fv_last_error())
    return status


def fv_patch_batch_update(patches_in, patches_out, sizes, offsets, num_patches: int, dim: int, unknowns: int,
                          dt: float, h: float, gamma: float = 1.4, flags: int = 0, lambda_out=None,
                          stream=None, raise_on_error: bool = True) -> int:
    """One explicit Euler step over a batch of patches; see include/fvpatch.h."""
    lib = load()
    sz, sz_p = _host_array(sizes, np.int32)
    of, of_p = _host_array(offsets, np.int64)
    st = lib.fv_patch_batch_update(_dev_ptr(patches_in), _dev_ptr(patches_out), sz_p, of_p, int(num_patches),
                                   int(dim), int(unknowns), float(dt), float(h), float(gamma), int(flags),
                                   _dev_ptr(lambda_out), _stream_handle(stream))
    del sz, of
    return _check(st) if raise_on_error else st


def fv_patch_batch_update_noalloc(patches_in, patches_out, sizes, offsets, num_patches: int, dim: int,
                                  unknowns: int, dt: float, h: float, gamma: float = 1.4, flags: int = 0,
                                  lambda_out=None, stream=None, raise_on_error: bool = True) -> int:
    """fv_patch_batch_update without any memory allocation in the library (fixed descriptor
    array, at most FV_NOALLOC_MAX_PATCHES patches); see include/fvpatch.h."""
    lib = load()
    sz, sz_p = _host_array(sizes, np.int32)
    of, of_p = _host_array(offsets, np.int64)
    st = lib.fv_patch_batch_update_noalloc(_dev_ptr(patches_in), _dev_ptr(patches_out), sz_p, of_p,
                                           int(num_patches), int(dim), int(unknowns), float(dt), float(h),
                                           float(gamma), int(flags), _dev_ptr(lambda_out), _stream_handle(stream))
    del sz, of
    return _check(st) if raise_on_error else st


def fv_set_tuning(dim: int, unknowns: int, p: int, tuning=None, raise_on_error: bool = True) -> int:
    """Install launch parameters for a patch class (a dict or fv_tuning; None restores defaults)."""
    lib = load()
    if tuning is None:
        st = lib.fv_set_tuning(int(dim), int(unknowns), int(p), None)
    else:
        t = tuning if isinstance(tuning, fv_tuning) else fv_tuning(**tuning)
        st = lib.fv_set_tuning(int(dim), int(unknowns), int(p), ctypes.byref(t))
    return _check(st) if raise_on_error else st


def fv_get_tuning(dim: int, unknowns: int, p: int) -> dict:
    """Launch parameters the library uses for a patch class."""
    lib = load()
    t = fv_tuning()
    _check(lib.fv_get_tuning(int(dim), int(unknowns), int(p), ctypes.byref(t)))
    return t.as_dict()


# ---------------------------------------------------------------- plans (batching form)
class fv_tune_entry(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("unknowns", ctypes.c_int32), ("p", ctypes.c_int32), ("tuning", fv_tuning)]


def tune_table(entries) -> ctypes.Array | None:
    """A plan's tuning table from {(dim, unknowns, p): {kernel, block, prefetch, rows}} (or a list of
    (dim, unknowns, p, dict) tuples); None for no entries."""
    items = list(entries.items()) if isinstance(entries, dict) else [((d, n, p), t) for d, n, p, t in entries]
    if not items:
        return None
    arr = (fv_tune_entry * len(items))()
    for k, ((d, n, p), t) in enumerate(items):
        tt = t if isinstance(t, fv_tuning) else fv_tuning(**{f: int(t.get(f, 0)) for f in ("kernel", "block",
                                                                                            "prefetch", "rows")})
        arr[k] = fv_tune_entry(int(d), int(n), int(p), tt)
    return arr


def fv_plan_create(sizes, offsets, num_patches: int, dim: int, unknowns: int, flags: int = 0, tune=None,
                   raise_on_error: bool = True):
    """Build a plan; returns its handle (an int), or (status, None) when raise_on_error is False.
    tune: the plan's own tuning table (see tune_table), or None."""
    lib = load()
    h = ctypes.c_void_p()
    sz, sz_p = _host_array(sizes, np.int32)
    of, of_p = _host_array(offsets, np.int64)
    table = tune_table(tune) if tune is not None else None
    st = lib.fv_plan_create(ctypes.byref(h), sz_p, of_p, int(num_patches), int(dim), int(unknowns), int(flags),
                            table, len(table) if table is not None else 0)
    del sz, of
    if raise_on_error:
        _check(st)
        return h.value
    return st, h.value


def fv_plan_get_tuning(plan, p: int) -> dict:
    t = fv_tuning()
    _check(load().fv_plan_get_tuning(plan, int(p), ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in fv_tuning._fields_}


def fv_plan_execute(plan, patches_in, patches_out, dt: float, h: float, gamma: float = 1.4, lambda_out=None,
                    stream=None, dt_dev=None, raise_on_error: bool = True) -> int:
    """One step of the plan; dt_dev (a device double) replaces the host dt when given."""
    st = load().fv_plan_execute(plan, _dev_ptr(patches_in), _dev_ptr(patches_out), float(dt), _dev_ptr(dt_dev),
                                float(h), float(gamma), _dev_ptr(lambda_out), _stream_handle(stream))
    return _check(st) if raise_on_error else st


def fv_plan_capture_steps(plan, steps: int, buf_a, buf_b, h: float, gamma: float, cfl: float, lambda_out, dt_dev,
                          stream=None, raise_on_error: bool = True) -> int:
    st = load().fv_plan_capture_steps(plan, int(steps), _dev_ptr(buf_a), _dev_ptr(buf_b), float(h), float(gamma),
                                      float(cfl), _dev_ptr(lambda_out), _dev_ptr(dt_dev), _stream_handle(stream))
    return _check(st) if raise_on_error else st


def fv_plan_replay(plan, stream=None, raise_on_error: bool = True) -> int:
    st = load().fv_plan_replay(plan, _stream_handle(stream))
    return _check(st) if raise_on_error else st


def fv_plan_info(plan) -> dict:
    info = fv_plan_stats()
    _check(load().fv_plan_info(plan, ctypes.byref(info)))
    return info.as_dict()


def fv_plan_destroy(plan) -> int:
    return _check(load().fv_plan_destroy(plan))


# ---------------------------------------------------------------- patch meshes (halo fill, local time stepping)
def fv_mesh_create(sizes, offsets, neighbors, num_patches: int, dim: int, unknowns: int,
                   raise_on_error: bool = True):
    """Build a mesh (neighbors: host [num_patches, 2*dim]); returns its handle, or
    (status, None) when raise_on_error is False."""
    lib = load()
    h = ctypes.c_void_p()
    sz, sz_p = _host_array(sizes, np.int32)
    of, of_p = _host_array(offsets, np.int64)
    nb, nb_p = _host_array(neighbors, np.int32)
    st = lib.fv_mesh_create(ctypes.byref(h), sz_p, of_p, nb_p, int(num_patches), int(dim), int(unknowns))
    del sz, of, nb
    if raise_on_error:
        _check(st)
        return h.value
    return st, h.value


def fv_mesh_halo_fill(mesh, patches, stream=None, raise_on_error: bool = True) -> int:
    st = load().fv_mesh_halo_fill(mesh, _dev_ptr(patches), _stream_handle(stream))
    return _check(st) if raise_on_error else st


def fv_mesh_step(mesh, patches_in, patches_out, dt, h, gamma: float = 1.4, lambda_out=None, stream=None,
                 raise_on_error: bool = True) -> int:
    st = load().fv_mesh_step(mesh, _dev_ptr(patches_in), _dev_ptr(patches_out), _dev_ptr(dt), _dev_ptr(h),
                             float(gamma), _dev_ptr(lambda_out), _stream_handle(stream))
    return _check(st) if raise_on_error else st


def fv_local_dt(lam, h, num_patches: int, dim: int, cfl: float, dt_out, stream=None,
                raise_on_error: bool = True) -> int:
    st = load().fv_local_dt(_dev_ptr(lam), _dev_ptr(h), int(num_patches), int(dim), float(cfl), _dev_ptr(dt_out),
                            _stream_handle(stream))
    return _check(st) if raise_on_error else st


def fv_mesh_destroy(mesh) -> int:
    return _check(load().fv_mesh_destroy(mesh))


# ---------------------------------------------------------------- the paper's realisations (comparison)
def fv_flavour_update(flavour: int, patches_in, patches_out, sizes, offsets, num_patches: int, dim: int,
                      unknowns: int, dt: float, h: float, gamma: float = 1.4, flags: int = 0, lambda_out=None,
                      stream=None, raise_on_error: bool = True) -> int:
    sz, sz_p = _host_array(sizes, np.int32)
    of, of_p = _host_array(offsets, np.int64)
    st = load().fv_flavour_update(int(flavour), _dev_ptr(patches_in), _dev_ptr(patches_out), sz_p, of_p,
                                  int(num_patches), int(dim), int(unknowns), float(dt), float(h), float(gamma),
                                  int(flags), _dev_ptr(lambda_out), _stream_handle(stream))
    del sz, of
    return _check(st) if raise_on_error else st


# ---------------------------------------------------------------- other PDEs (the generic solver)
def fv_pde_unknowns(pde: int, dim: int) -> tuple[int, int]:
    """(unknowns per volume, number of parameters) of a built-in PDE."""
    nq, npr = ctypes.c_int32(), ctypes.c_int32()
    _check(load().fv_pde_unknowns(int(pde), int(dim), ctypes.byref(nq), ctypes.byref(npr)))
    return nq.value, npr.value


def fv_pde_batch_update(pde: int, params, patches_in, patches_out, sizes, offsets, num_patches: int, dim: int,
                        dt: float, h: float, flags: int = 0, lambda_out=None, stream=None,
                        raise_on_error: bool = True) -> int:
    """One explicit Euler step of every patch for the PDE `pde` (see include/fvpatch.h)."""
    pr, pr_p = _host_array(params, np.float64)
    sz, sz_p = _host_array(sizes, np.int32)
    of, of_p = _host_array(offsets, np.int64)
    st = load().fv_pde_batch_update(int(pde), pr_p, 0 if pr is None else len(pr), _dev_ptr(patches_in),
                                    _dev_ptr(patches_out), sz_p, of_p, int(num_patches), int(dim), float(dt),
                                    float(h), int(flags), _dev_ptr(lambda_out), _stream_handle(stream))
    del pr, sz, of
    return _check(st) if raise_on_error else st


# ---------------------------------------------------------------- patches in host memory
def host_pointer_table(patches) -> np.ndarray:
    """Host addresses of a sequence of numpy float64 arrays (C-contiguous), as the
    pointer table fv_host_patches_update takes; the arrays must outlive its use."""
    addrs = np.empty(len(patches), np.uintp)
    for t, a in enumerate(patches):
        if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous:
            raise ValueError(f"patch {t} must be a C-contiguous float64 numpy array")
        addrs[t] = a.ctypes.data
    return addrs


def fv_host_alloc(nbytes: int, raise_on_error: bool = True):
    """Pinned host memory for zero-copy patches: returns its address (int)."""
    p = ctypes.c_void_p()
    st = load().fv_host_alloc(int(nbytes), ctypes.byref(p))
    if raise_on_error:
        _check(st)
        return p.value
    return st, p.value


def fv_host_free(addr, raise_on_error: bool = True) -> int:
    st = load().fv_host_free(addr)
    return _check(st) if raise_on_error else st


def pinned_array(addr: int, n: int) -> np.ndarray:
    """A float64 numpy view of n doubles at `addr` (memory from fv_host_alloc); the view
    must not be used after fv_host_free."""
    return np.ctypeslib.as_array((ctypes.c_double * n).from_address(addr))


def fv_host_patches_update(patches_in, patches_out, sizes, num_patches: int, dim: int, unknowns: int, dt: float,
                           h: float, gamma: float = 1.4, flags: int = 0, lambda_out=None, config=None, stats=None,
                           raise_on_error: bool = True) -> int:
    """One step of patches held in host memory (see include/fvpatch.h).  patches_in /
    patches_out: sequences of float64 numpy arrays, or uintp tables of host addresses
    (host_pointer_table); lambda_out: float64 numpy array or None; config: a dict of
    fv_transfer_config fields or None; stats: a dict filled with fv_transfer_stats."""
    def table(x, writable):
        if isinstance(x, np.ndarray) and x.dtype == np.uintp:
            return x
        if writable and any(not a.flags.writeable for a in x):
            raise ValueError("output patches must be writable")
        return host_pointer_table(x)
    tin, tout = table(patches_in, False), table(patches_out, True)
    if len(tin) < num_patches or len(tout) < num_patches:
        raise ValueError("fewer patch pointers than num_patches")
    sz, sz_p = _host_array(sizes, np.int32)
    lam_p = None
    if lambda_out is not None:
        if not isinstance(lambda_out, np.ndarray) or lambda_out.dtype != np.float64 or \
                not lambda_out.flags.c_contiguous or lambda_out.size < num_patches:
            raise ValueError("lambda_out must be a contiguous float64 numpy array of num_patches entries")
        lam_p = lambda_out.ctypes.data
    cfg = None
    if config is not None:
        cfg = fv_transfer_config(**config) if isinstance(config, dict) else config
    st_out = fv_transfer_stats()
    st = load().fv_host_patches_update(tin.ctypes.data, tout.ctypes.data, sz_p, int(num_patches), int(dim),
                                       int(unknowns), float(dt), float(h), float(gamma), int(flags), lam_p,
                                       ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(st_out))
    del sz
    if stats is not None:
        stats.update(st_out.as_dict())
    return _check(st) if raise_on_error else st


# ---------------------------------------------------------------- servers (serving form)
def fv_server_create(budget_bytes: int, gamma: float = 1.4, flags: int = 0, mode: int = 0, max_inflight: int = 0,
                     max_retries: int = 0, deadline_ms: float = 0.0, raise_on_error: bool = True):
    cfg = fv_server_config(int(budget_bytes), float(gamma), int(flags), int(mode), int(max_inflight),
                           int(max_retries), float(deadline_ms))
    hdl = ctypes.c_void_p()
    st = load().fv_server_create(ctypes.byref(hdl), ctypes.byref(cfg))
    if raise_on_error:
        _check(st)
        return hdl.value
    return st, hdl.value


def fv_server_add_mesh(server, dim: int, unknowns: int, h: float, sizes, host_state, raise_on_error: bool = True):
    """Register a mesh (host_state: float64 array in the contiguous layout); returns its id."""
    sz, sz_p = _host_array(sizes, np.int32)
    state = np.ascontiguousarray(host_state, dtype=np.float64)
    mid = ctypes.c_int32(-1)
    st = load().fv_server_add_mesh(server, int(dim), int(unknowns), float(h), sz_p, len(sz), state.ctypes.data,
                                   ctypes.byref(mid))
    del sz
    if raise_on_error:
        _check(st)
        return mid.value
    return st, mid.value


def fv_server_inject(server, ticket: int, kind: int, times: int = 0, raise_on_error: bool = True) -> int:
    """Test hook: override the completion check of batch `ticket` (FV_INJECT_FAIL / FV_INJECT_HANG; 0 clears)."""
    st = load().fv_server_inject(server, int(ticket), int(kind), int(times))
    return _check(st) if raise_on_error else st


def fv_server_batch_log(server) -> np.ndarray:
    """Records of the completed batches (structured array of BATCH_RECORD_DTYPE)."""
    n = ctypes.c_int64(0)
    _check(load().fv_server_batch_log(server, None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=BATCH_RECORD_DTYPE)
    if n.value:
        _check(load().fv_server_batch_log(server, out.ctypes.data, n.value, ctypes.byref(n)))
    return out


def fv_server_submit(server, mesh: int, first: int, count: int, dt: float, arrival_ns: int = 0,
                     raise_on_error: bool = True):
    ticket = ctypes.c_int64(0)
    st = load().fv_server_submit(server, int(mesh), int(first), int(count), float(dt), int(arrival_ns),
                                 ctypes.byref(ticket))
    if raise_on_error:
        _check(st)
        return ticket.value
    return st


def _stats_call(fn, server, raise_on_error=True):
    out = fv_server_stats()
    st = fn(server, ctypes.byref(out))
    if raise_on_error:
        _check(st)
        return out.as_dict()
    return st, out.as_dict()


def fv_server_poll(server, raise_on_error: bool = True):
    return _stats_call(load().fv_server_poll, server, raise_on_error)


def fv_server_drain(server, raise_on_error: bool = True):
    return _stats_call(load().fv_server_drain, server, raise_on_error)


def fv_server_stats_get(server):
    return _stats_call(load().fv_server_stats_get, server)


def fv_server_run_trace(server, requests: np.ndarray, raise_on_error: bool = True):
    """requests: structured array of SERVE_REQUEST_DTYPE (arrival_ns relative to the start)."""
    req = np.ascontiguousarray(requests, dtype=SERVE_REQUEST_DTYPE)
    out = fv_server_stats()
    st = load().fv_server_run_trace(server, req.ctypes.data, len(req), ctypes.byref(out))
    if raise_on_error:
        _check(st)
        return out.as_dict()
    return st, out.as_dict()


def fv_server_read_mesh(server, mesh: int, out: np.ndarray) -> np.ndarray:
    assert out.dtype == np.float64 and out.flags.c_contiguous
    _check(load().fv_server_read_mesh(server, int(mesh), out.ctypes.data))
    return out


def fv_server_destroy(server) -> int:
    return _check(load().fv_server_destroy(server))
