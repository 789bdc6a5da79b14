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
import sys
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


def run(mode: int, meshes, trace: np.ndarray, budget: int = BUDGET_BYTES, max_inflight: int = 8,
        read_back: bool = False, h: float = wl.H_DEFAULT, flags: int = fv.FV_HALO_PERIODIC):
    """Replay a trace over one or several meshes (trace["mesh"] indexes `meshes`; each mesh keeps
    its own dimension) in ONE fresh server: one stream, one resident pool, one budget.  Returns
    (stats, batch log, [final state per mesh] or None)."""
    if isinstance(meshes, wl.Batch):
        meshes = [meshes]
    srv = fv.fv_server_create(budget, wl.GAMMA, flags, mode, max_inflight)
    try:
        ids = [fv.fv_server_add_mesh(srv, m.dim, m.nq, h, m.sizes, m.data) for m in meshes]
        assert ids == list(range(len(meshes)))
        st = fv.fv_server_run_trace(srv, trace)
        log = fv.fv_server_batch_log(srv)
        states = [fv.fv_server_read_mesh(srv, i, np.empty_like(m.data)) for i, m in zip(ids, meshes)] \
            if read_back else None
        return st, log, states
    finally:
        fv.fv_server_destroy(srv)


def latency_summary(log: np.ndarray, select=None) -> dict:
    """p50 / p99 / max / mean of arrival-to-completion latency (ms) over the records `select`
    picks, with the queueing part (arrival to launch) and the rest (launch to completion seen)."""
    r = log if select is None else log[select]
    if len(r) == 0:
        return {"batches": 0}
    lat = (r["done_ns"] - r["arrival_ns"]) * 1e-6
    wait = (r["launch_ns"] - r["arrival_ns"]) * 1e-6
    run_ = (r["done_ns"] - r["launch_ns"]) * 1e-6
    q = lambda a, x: round(float(np.percentile(a, x)), 4)  # noqa: E731
    return {"batches": int(len(r)), "p50_ms": q(lat, 50), "p99_ms": q(lat, 99), "max_ms": round(float(lat.max()), 4),
            "mean_ms": round(float(lat.mean()), 4), "queue_p50_ms": q(wait, 50), "queue_p99_ms": q(wait, 99),
            "launch_to_done_p50_ms": q(run_, 50), "launch_to_done_p99_ms": q(run_, 99),
            "cells": int(r["cells"].sum())}


def bench_main(args) -> int:
    """bench.py --form serving: config 5, one Poisson stream of 2D mixed and 3D 8^3 batches (4:1) through
    ONE server holding both meshes under the 64 GB budget, once with the fused loop and once with the
    plain per-batch loop, on the same trace.  One JSON line per mode."""
    seconds = float(args.serve_seconds)
    rate = 2000.0
    patches_2d, patches_3d = 500_000, 50_000
    t_build = time.perf_counter()
    m2, m3 = build_meshes(patches_2d, patches_3d, seed=args.seed)
    t_build = time.perf_counter() - t_build
    trace = make_trace(rate, seconds, [patches_2d, patches_3d], seed=args.seed)
    res = {}
    print(f"serving: meshes built in {t_build:.1f} s, trace of {len(trace)} batches over {seconds:.0f} s",
          file=sys.stderr, flush=True)
    for mode, name in ((fv.FV_SERVE_FUSED, "fused"), (fv.FV_SERVE_PLAIN, "plain")):
        st, log, _ = run(mode, [m2, m3], trace)
        res[name] = (st, log)
        print(f"serving: {name} replay done ({st['completed']} batches)", file=sys.stderr, flush=True)
    for name, (st, log) in res.items():
        other = "plain" if name == "fused" else "fused"
        overall = latency_summary(log)
        line = {"metric": "p50/p99 batch latency (arrival to completion) and cell-updates/s",
                "form": "serving", "mode": name, "p50_ms": overall["p50_ms"], "p99_ms": overall["p99_ms"],
                "max_ms": overall["max_ms"], "mean_ms": overall["mean_ms"],
                "value": round(st["cell_updates_per_s"], 1), "unit": "cell-updates/s",
                "batches": st["completed"], "submitted": st["submitted"], "failed": st["failed"],
                "peak_queued": st["peak_queued"], "peak_inflight": st["peak_inflight"],
                "resident_GB": round(st["resident_bytes"] / 1e9, 3), "budget_GB": round(st["budget_bytes"] / 1e9, 1),
                "overall": overall,
                "by_class": {"2d_mixed": latency_summary(log, log["mesh"] == 0),
                             "3d_8cubed": latency_summary(log, log["mesh"] == 1)},
                f"p99_vs_{other}": round(overall["p99_ms"] / latency_summary(res[other][1])["p99_ms"], 3),
                "dtype": "f64", "data": "synthetic",
                "config": {"workload": "c5_serving_mixed_stream", "rate_per_s": rate, "seconds": seconds,
                           "batch_patches": "U{1..4096}", "meshes": {"2d_mixed_3_5_9_17": patches_2d,
                                                                      "3d_p8": patches_3d},
                           "class_weights": "2D:3D = 4:1", "servers": 1, "max_inflight": 8},
                "mesh_build_s": round(t_build, 1)}
        print(json.dumps(line), flush=True)
    return 0
