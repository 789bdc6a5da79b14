"""Serving form: seeded request traces and the serving benchmark (config 5).

Trace recipe (the paper fixes none; this stands in for the batches a mesh
traversal would emit, Sec. 2.1): Poisson arrivals with mean rate `rate`
batches/s for `seconds`; batch size U{1..4096} patches; each batch belongs to
the 2D mesh (mixed sizes {3, 5, 9, 17}) or the 3D mesh (8^3), 4:1; a batch is
the next contiguous range of its mesh in traversal order, wrapping to the
start (a batch that would run past the end stops there).  Draw order with
numpy PCG64(seed): arrival gaps, sizes, classes.
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import fvpatch as fv
from . import workloads as wl

BUDGET_BYTES = 64 << 30


def make_trace(rate: float, seconds: float, mesh_patches: list[int], weights=(4, 1), max_batch: int = 4096,
               dt=(1e-4, 1e-4), seed: int = 0) -> np.ndarray:
    """Structured array of fv.SERVE_REQUEST_DTYPE.  dt[m]: step size of mesh m."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rate * seconds * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps)
    n = int(np.searchsorted(arrivals, seconds))
    arrivals = arrivals[:n]
    counts = rng.integers(1, max_batch + 1, n)
    w = np.asarray(weights, float)
    cls = rng.choice(len(mesh_patches), size=n, p=w / w.sum())
    req = np.zeros(n, dtype=fv.SERVE_REQUEST_DTYPE)
    pos = [0] * len(mesh_patches)
    for k in range(n):
        m = int(cls[k])
        M = mesh_patches[m]
        c = int(min(counts[k], M - pos[m]))
        req[k] = (int(arrivals[k] * 1e9), m, pos[m], c, 0, dt[m])
        pos[m] = (pos[m] + c) % M
    return req


def build_meshes(patches_2d: int, patches_3d: int, seed: int = 0):
    """Host states of the two meshes: 2D mixed {3,5,9,17} (N=5) and 3D 8^3 (N=5)."""
    m2 = wl.make_mixed(patches_2d, (3, 5, 9, 17), dim=2, nq=5, seed=seed)
    m3 = wl.make_uniform(patches_3d, 8, dim=3, nq=5, seed=seed + 1)
    return m2, m3


def run(mode: int, mesh: wl.Batch, trace: np.ndarray, budget: int = BUDGET_BYTES, max_inflight: int = 8,
        read_back: bool = False):
    """Replay a trace over one mesh (trace["mesh"] must be 0) in a fresh server; returns (stats, final state or None)."""
    srv = fv.fv_server_create(budget, mesh.dim, mesh.nq, wl.H_DEFAULT, wl.GAMMA, fv.FV_HALO_PERIODIC, mode,
                              max_inflight)
    try:
        mid = fv.fv_server_add_mesh(srv, mesh.sizes, mesh.data)
        t = trace.copy()
        t["mesh"] = mid
        st = fv.fv_server_run_trace(srv, t)
        state = fv.fv_server_read_mesh(srv, mid, np.empty_like(mesh.data)) if read_back else None
        return st, state
    finally:
        fv.fv_server_destroy(srv)


def bench_main(args) -> int:
    """bench.py --form serving: config 5 through the fused loop and the plain per-batch loop."""
    seconds = float(args.serve_seconds)
    rate = 2000.0
    patches_2d, patches_3d = 500_000, 50_000
    t_build = time.perf_counter()
    m2, m3 = build_meshes(patches_2d, patches_3d, seed=args.seed)
    t_build = time.perf_counter() - t_build
    trace = make_trace(rate, seconds, [patches_2d, patches_3d], seed=args.seed)
    for mode, name in ((fv.FV_SERVE_FUSED, "fused"), (fv.FV_SERVE_PLAIN, "plain")):
        res = {}
        for dim, mesh_index, b in ((2, 0, m2), (3, 1, m3)):
            t = trace[trace["mesh"] == mesh_index].copy()
            t["mesh"] = 0
            res[dim], _ = run(mode, b, t)
        for dim, st in res.items():
            line = {"metric": "p50/p99 batch latency (arrival to completion) and cell-updates/s",
                    "form": "serving", "mode": name, "mesh": "2D mixed {3,5,9,17}^2" if dim == 2 else "3D 8^3",
                    "p50_ms": round(st["p50_ms"], 4), "p99_ms": round(st["p99_ms"], 4), "max_ms": round(st["max_ms"], 4),
                    "mean_ms": round(st["mean_ms"], 4), "value": round(st["cell_updates_per_s"], 1),
                    "unit": "cell-updates/s", "batches": st["completed"], "peak_queued": st["peak_queued"],
                    "peak_inflight": st["peak_inflight"], "resident_GB": round(st["resident_bytes"] / 1e9, 3),
                    "budget_GB": round(st["budget_bytes"] / 1e9, 1), "dtype": "f64", "data": "synthetic",
                    "config": {"workload": "c5_serving", "rate_per_s": rate, "seconds": seconds,
                               "batch_patches": "U{1..4096}", "meshes": {"2d": patches_2d, "3d": patches_3d},
                               "class_weights": "2D:3D = 4:1"},
                    "mesh_build_s": round(t_build, 1)}
            print(json.dumps(line), flush=True)
    return 0
