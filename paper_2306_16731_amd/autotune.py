"""Autotuner for the patch-update launches (batching form).

For every patch class (dim, unknowns, p) it times candidate launch parameters
-- kernel (2D wave kernel built for the size / 2D wave / 2D tile /
plane-marching block kernel), threads per block, rows of load prefetch,
output rows staged per burst -- on a synthetic
batch of that class, ping-ponging steps through the C ABI after a warmup,
and installs the fastest with fv_set_tuning.  Plans built afterwards pick the
installed parameters up per size class.  For a whole batch it also picks the
plan's launch mode: the fused launch on a persistent grid walking the task
list, the fused launch with one wave per task, or one launch per size class.

The table persists as JSON:

    {"device": "...", "entries": {"2,5,16": {"kernel": 2, "block": 256, "prefetch": 4, "rows": 6,
                                             "ms": 0.37, "patches": 65536}, ...},
     "plans": {"<composition key>": {"mode": "per_class", "flags": 512, "ms": ...}}}
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import fvpatch as fv
from . import workloads as wl

TARGET_CELLS = 1 << 24  # cells per timed step: the size of the benchmark batches, far above the caches
MAX_PATCHES = 1 << 18   # ... but at most this many patches (small sizes: host-side generation time)


def class_key(dim: int, nq: int, p: int) -> str:
    return f"{dim},{nq},{p}"


def candidates(dim: int, nq: int, p: int) -> list[dict]:
    """Launch parameters worth timing for a class (the library rejects ones that do not fit)."""
    out = []
    if nq == 5 and p in (fv.FIXED_SIZES_2D if dim == 2 else fv.FIXED_SIZES_3D):
        out.append(dict(kernel=fv.FV_KERNEL_FIXED, block=0, prefetch=0, rows=0))
    if dim == 2 and p + 2 <= 64:
        for pf in (2, 3, 4):
            for rows in (4, 6, 8):
                for blk in (128, 256):
                    out.append(dict(kernel=fv.FV_KERNEL_WAVE, block=blk, prefetch=pf, rows=rows))
    if dim == 2 and p * p <= 1024:
        c = p * p
        blocks = sorted({max(64, ((c + 63) // 64) * 64), 256} | ({512} if c <= 512 else set()))
        for blk in blocks:
            if blk >= c and blk <= 1024:
                out.append(dict(kernel=fv.FV_KERNEL_TILE, block=blk, prefetch=0, rows=0))
    lanes = (p + 2) if dim == 2 else (p + 2) ** 2
    for blk in range(64, 1025, 64):
        if blk < lanes:
            continue
        util = (blk // lanes) * lanes / blk
        if util >= 0.75:
            out.append(dict(kernel=fv.FV_KERNEL_BLOCK, block=blk, prefetch=0, rows=0))
        if len([c for c in out if c["kernel"] == fv.FV_KERNEL_BLOCK]) >= 4:
            break
    return out


def _time_steps(step, steps: int, warmup: int) -> float:
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


class ClassBatch:
    """A synthetic batch of one class, resident on the device, reused by every candidate."""

    def __init__(self, dim: int, nq: int, p: int, seed: int = 0):
        import torch
        self.dim, self.nq, self.p = dim, nq, p
        self.T = min(MAX_PATCHES, max(256, TARGET_CELLS // p ** dim))
        b = wl.make_uniform(self.T, p, dim=dim, nq=nq, seed=seed)
        self.sizes = b.sizes
        self.bufs = [torch.from_numpy(b.data).to("cuda"), None]
        self.bufs[1] = self.bufs[0].clone()
        self.lam = torch.empty(self.T, dtype=torch.float64, device="cuda")


def time_class(batch: ClassBatch, tuning: dict | None, steps: int = 10, warmup: int = 20,
               periodic: bool = False) -> float | None:
    """ms per plain-launch step of the class batch under `tuning`; None if the tuning is rejected."""
    b = batch
    st = fv.fv_set_tuning(b.dim, b.nq, b.p, tuning, raise_on_error=False)
    if st != fv.FV_OK:
        return None
    flags = fv.FV_HALO_PERIODIC if periodic else 0

    def step():
        fv.fv_patch_batch_update(b.bufs[0], b.bufs[1], b.sizes, None, b.T, b.dim, b.nq, 1e-3, wl.H_DEFAULT,
                                 wl.GAMMA, flags, b.lam)
        b.bufs.reverse()

    try:
        return _time_steps(step, steps, warmup)
    except fv.FvError:
        return None


def tune_class(dim: int, nq: int, p: int, verbose: bool = False, periodic: bool = False) -> dict:
    """Time every candidate of a class (with or without periodic face halos, as the
    workload runs), install and return the fastest."""
    best = None
    batch = ClassBatch(dim, nq, p)
    for cand in candidates(dim, nq, p):
        ms = time_class(batch, cand, periodic=periodic)
        if verbose:
            print(f"  {dim}D N={nq} p={p} {cand} -> {ms}", flush=True)
        if ms is not None and (best is None or ms < best["ms"]):
            best = dict(cand, ms=ms)
    if best is None:
        fv.fv_set_tuning(dim, nq, p, None)
        return {}
    fv.fv_set_tuning(dim, nq, p, {k: best[k] for k in ("kernel", "block", "prefetch", "rows")})
    best["patches"] = batch.T
    del batch
    import torch
    torch.cuda.empty_cache()
    return best


def tune_classes(classes, verbose: bool = False, periodic: bool = False) -> dict:
    """classes: iterable of (dim, nq, p).  Returns {key: best}."""
    return {class_key(*c): tune_class(*c, verbose=verbose, periodic=periodic) for c in classes}


def plan_table(entries: dict) -> dict:
    """A plan's own tuning table ({(dim, nq, p): tuning}, for fv_plan_create's `tune`) from the
    entries of tune_classes or of a saved table."""
    out = {}
    for key, e in entries.items():
        if not e:
            continue
        dim, nq, p = (int(x) for x in key.split(","))
        out[(dim, nq, p)] = {k: int(e[k]) for k in ("kernel", "block", "prefetch", "rows")}
    return out


def composition_key(sizes, dim: int, nq: int) -> str:
    vals, counts = np.unique(np.asarray(sizes), return_counts=True)
    return f"{dim},{nq}:" + ";".join(f"{int(v)}x{int(c)}" for v, c in zip(vals, counts))


PLAN_MODES = {"persistent": 0, "per_task": fv.FV_PLAN_NO_PERSIST, "per_class": fv.FV_PLAN_PER_CLASS}


def tune_plan(batch: wl.Batch, periodic: bool = False, steps: int = 10, warmup: int = 10, tune=None) -> dict:
    """The plan's launch mode for a batch composition, by timing: the fused launch on a persistent
    grid, the fused launch with one wave per task, or one launch per size class (each plan with the
    tuning table `tune`, if given).  Returns {"mode", "flags", "ms", "ms_<mode>" for each mode}."""
    import torch
    res = {}
    for mode, mflags in PLAN_MODES.items():
        flags = (fv.FV_HALO_PERIODIC if periodic else 0) | mflags
        plan = fv.fv_plan_create(batch.sizes, batch.offsets, batch.num_patches, batch.dim, batch.nq, flags, tune=tune)
        try:
            a = torch.from_numpy(batch.data).to("cuda")
            c = a.clone()
            lam = torch.empty(batch.num_patches, dtype=torch.float64, device="cuda")
            bufs = [a, c]

            def step():
                fv.fv_plan_execute(plan, bufs[0], bufs[1], 1e-3, wl.H_DEFAULT, wl.GAMMA, lam)
                bufs.reverse()

            res[mode] = _time_steps(step, steps, warmup)
            del a, c, lam
        finally:
            fv.fv_plan_destroy(plan)
    best = min(res, key=res.get)
    return {"mode": best, "flags": PLAN_MODES[best], "ms": res[best], **{f"ms_{m}": t for m, t in res.items()}}


def device_name() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "none"


def save(table: dict, path: str) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path: str, install: bool = True) -> dict:
    """Read a table; install its entries with fv_set_tuning (unless install=False)."""
    with open(path) as f:
        table = json.load(f)
    if install:
        for key, e in table.get("entries", {}).items():
            if not e:
                continue
            dim, nq, p = (int(x) for x in key.split(","))
            fv.fv_set_tuning(dim, nq, p, {k: e[k] for k in ("kernel", "block", "prefetch", "rows")})
    return table


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description="tune patch-update launches for the given classes")
    ap.add_argument("--classes", default="2,5,3;2,5,5;2,5,9;2,5,16;2,5,17;3,5,8",
                    help="semicolon-separated dim,unknowns,p triples")
    ap.add_argument("--out", default=None, help="write the table here (JSON)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--periodic", action="store_true", help="tune with periodic face halos")
    args = ap.parse_args(argv)
    fv.load()
    classes = [tuple(int(x) for x in c.split(",")) for c in args.classes.split(";") if c]
    t0 = time.perf_counter()
    entries = tune_classes(classes, verbose=args.verbose, periodic=args.periodic)
    table = {"device": device_name(), "seconds": round(time.perf_counter() - t0, 2), "entries": entries}
    print(json.dumps(table), flush=True)
    if args.out:
        save(table, args.out)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
