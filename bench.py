#!/usr/bin/env python3
"""Benchmark of the FV patch update on one MI355X.

Default workload: 65536 patches of 16 x 16 interior volumes (18 x 18 x 5
doubles each, AoS per volume), 2D compressible Euler, Rusanov flux, FP64,
seeded rho/u/v/w/p draws plus a Gaussian density pulse per patch, periodic
face-halo write and the per-patch eigenvalue reduction, as one
fv_patch_batch_update call per time step.  A "step" is one such call over the
whole batch (one explicit Euler time step of every patch).

Prints ONE JSON line with the metric (cell-updates/s over the timed steps,
inputs resident in HBM), the roofline of the update kernel (algorithmic bytes
per launch / average launch time, against 8 TB/s), and the CPU oracle timed on
a bounded sample of the same workload on the host's cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources of the kernel the roofline reports (the 2D wave kernel and its physics)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2306_16731_amd", "csrc", f) for f in ("fv_update2d.hip", "fv_physics.h", "fv_pde.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fv_update_c2_2d_p16_T65536_traffic.md")


def alg_bytes_per_patch(p: int, dim: int, nq: int, periodic: bool, with_lambda: bool) -> int:
    """Bytes the method must move per patch: the face-halo-padded input (corner / edge
    halo volumes excluded), the interior output, the periodic face-halo output, lambda."""
    inner = p ** dim
    faces = 2 * dim * p ** (dim - 1)
    read = (inner + faces) * nq * 8
    write = inner * nq * 8 + (faces * nq * 8 if periodic else 0)
    return read + write + (8 if with_lambda else 0)


KERNEL_LABELS = {1: "update_kernel (plane-marching block kernel)", 2: "update2d_kernel (2D wave kernel, runtime size)",
                 3: "update2d_tile_kernel (2D tile kernel)",
                 4: "update2d_fixed_kernel (2D wave kernel built for the patch size)"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m_sha = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m_sha and m_b) or m_sha.group(1) != kernel_sha():
        return None
    return float(m_b.group(1))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed steps first (about 40 ms: the GPU's clocks and TLBs settle)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-patches", type=int, default=8192,
                    help="patches the CPU oracle advances through all warmup + timed steps")
    ap.add_argument("--form", choices=["plain", "batching", "serving", "mesh", "flavours", "transfer", "pde", "latency"],
                    default="plain",
                    help="plain: the headline line (config 2).  batching: configs 3 and 4 through plain launches, "
                         "plans and captured graphs (one line each).  serving: the request loop (config 5).  "
                         "latency: launch-to-done p50/p99 of config 1 (16 patches of 3^2, cache-resident)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the serving trace")
    ap.add_argument("--tuning-table", default=None, help="install this autotuner table instead of tuning now")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run 4 update launches and one 849,346,560-byte device copy, for rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE runs (the copy's reading is the counters' scale), then exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the patch update is measured on a "
              "single MI355X; sharding across GPUs is described in DESIGN.md, not run.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    fvpatch.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.form == "mesh":
        return bench_mesh(args)
    if args.form == "flavours":
        return bench_flavours(args)
    if args.form == "transfer":
        return bench_transfer(args)
    if args.form == "pde":
        return bench_pde(args)
    if args.form == "batching":
        return bench_batching(args)
    if args.form == "latency":
        return bench_latency(args)
    if args.form == "serving":
        from paper_2306_16731_amd import serving
        return serving.bench_main(args)
    dev = torch.device("cuda:0")
    name = "c2_2d_p16_T65536"
    b, spec = wl.build_workload(name, seed=args.seed)
    T, p, dim, nq = b.num_patches, int(b.sizes[0]), b.dim, b.nq
    periodic = spec["periodic"]
    flags = fvpatch.FV_HALO_PERIODIC if periodic else 0
    h, gamma = wl.H_DEFAULT, wl.GAMMA

    d_a = torch.from_numpy(b.data).to(dev)
    d_b = d_a.clone()
    lam = torch.empty(T, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    if args.traffic_probe:
        for _ in range(4):
            fvpatch.fv_patch_batch_update(d_a, d_b, b.sizes, None, T, dim, nq, 1.6e-3, h, gamma, flags, lam, stream)
        d_b.copy_(d_a)  # plain copy of known size: d_a.numel() * 8 bytes read and written
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": d_a.numel() * 8, "kernel_sources_sha": kernel_sha()}))
        return 0

    # time step from the initial eigenvalue (outside the timed region)
    fvpatch.fv_patch_batch_update(d_a, d_b, b.sizes, None, T, dim, nq, 1e-9, h, gamma, flags, lam, stream)
    torch.cuda.synchronize()
    dt = wl.CFL * h / (dim * float(lam.max().item()))
    d_b.copy_(d_a)

    def step(src, dst):
        fvpatch.fv_patch_batch_update(src, dst, b.sizes, None, T, dim, nq, dt, h, gamma, flags, lam, stream)

    for _ in range(args.warmup):
        step(d_a, d_b)
        d_a, d_b = d_b, d_a
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step(d_a, d_b)
        d_a, d_b = d_b, d_a
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    cells = T * p ** dim
    value = cells * args.steps / (gpu_ms / 1e3)

    # the oracle's sample is compared against the state right after the timed steps
    S = min(args.cpu_sample_patches, T)
    sample_state = d_a[: S * int(b.offsets[1])].clone()

    # the same K-step measurement repeated (median of 16 samples), then a plain device copy of the
    # state as the streaming ceiling of this GPU (sanity check of the roofline)
    samples = []
    for _ in range(16):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            step(d_a, d_b)
            d_a, d_b = d_b, d_a
        e1.record(stream)
        torch.cuda.synchronize()
        samples.append(e0.elapsed_time(e1) / args.steps)
    samples.sort()
    scratch = torch.empty_like(d_a)
    for _ in range(3):
        scratch.copy_(d_a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        scratch.copy_(d_a)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * d_a.numel() * 8 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del scratch

    per_launch = alg_bytes_per_patch(p, dim, nq, periodic, True) * T
    achieved = per_launch / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 4),
                "kernel": KERNEL_LABELS.get(fvpatch.fv_get_tuning(dim, nq, p)["kernel"], "?"),
                "alg_bytes_per_launch": per_launch,
                "alg_bytes_per_cell": round(per_launch / cells, 3),
                "torch_copy_GBs": round(copy_gbs, 1), "frac_of_torch_copy": round(achieved / copy_gbs, 4)}

    out = {
        "metric": "cell-updates/s", "value": round(value, 1), "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": name, "patches": T, "p": p, "dim": dim, "unknowns": nq, "periodic_halo": periodic,
                   "eigenvalue_reduction": True, "path": "fv_patch_batch_update", "dt": dt, "h": h},
        "dof_updates_per_s": round(value * nq, 1),
        "roofline": roofline,
        "host_wall_s": round(wall, 4),
        "repeat": {"samples": len(samples), "median_ms_per_step": round(samples[len(samples) // 2], 5),
                   "min_ms_per_step": round(samples[0], 5), "max_ms_per_step": round(samples[-1], 5)},
        "tuning": fvpatch.fv_get_tuning(dim, nq, p),
    }

    if not args.no_cpu_baseline:
        import oracle
        steps_total = args.warmup + args.steps
        sub = b.data[: S * int(b.offsets[1])]
        threads = oracle.max_threads()
        t0 = time.perf_counter()
        ora_state, _ = oracle.run_steps(sub, b.sizes[:S], b.offsets[:S], dim, nq, [dt] * steps_total, h, gamma,
                                        periodic, nthreads=threads)
        cpu_s = time.perf_counter() - t0
        # one thread on a smaller sample of the same patches and steps
        S1 = max(1, S // 16)
        t1 = time.perf_counter()
        oracle.run_steps(b.data[: S1 * int(b.offsets[1])], b.sizes[:S1], b.offsets[:S1], dim, nq, [dt] * steps_total,
                         h, gamma, periodic, nthreads=1)
        cpu1_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(S * p ** dim * steps_total / cpu_s, 1), "unit": "cell-updates/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"first {S} of the {T} patches, {steps_total} steps, same dt, "
                                         f"OpenMP over patches ({cpu_s:.2f} s wall)",
                               "single_thread": {"value": round(S1 * p ** dim * steps_total / cpu1_s, 1),
                                                 "sample": f"first {S1} patches, {steps_total} steps "
                                                           f"({cpu1_s:.2f} s wall)"},
                               "cpu_work_core_s": round(cpu_s * threads + cpu1_s, 1),
                               "host_cpus_visible": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}
        # the timed GPU run advanced the same patches with the same dt: compare them
        got = sample_state.cpu().numpy()
        g = got.reshape(-1, nq)
        w = ora_state.reshape(-1, nq)
        errs = np.max(np.abs(g - w), axis=0) / np.max(np.abs(w), axis=0)
        out["parity_sample"] = {"patches": S, "steps": steps_total, "max_rel_err": float(np.max(errs)),
                                "tolerance": 1e-12}
    print(json.dumps(out), flush=True)
    return 0


def _timed(fn, steps: int) -> float:
    """Seconds for `steps` calls of fn, bracketed by device synchronisation."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def bench_latency(args, samples: int = 4000) -> int:
    """Config 1 (16 patches of 3 x 3, 2D Euler, one step): 19 KB of state, so the step is bound by
    launch and completion latency, not by HBM.  For the plain call, a plan's fused launch and a
    one-step captured graph: host time from the call to the stream's completion, per sample
    (p50 / p99 / max), and the device time per launch when launches run back to back.  The plain call
    runs twice: with an offsets array (uploaded with the call) and contiguous (offsets NULL, nothing
    uploaded)."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    name = "c1_2d_p3_T16"
    b, spec = wl.build_workload(name, seed=args.seed)
    T, dim, nq = b.num_patches, b.dim, b.nq
    flags = fvpatch.FV_HALO_PERIODIC if spec["periodic"] else 0
    h, dt = wl.H_DEFAULT, 1.0e-3
    stream = torch.cuda.Stream()
    a = torch.from_numpy(b.data).to("cuda")
    c = a.clone()
    lam = torch.empty(T, dtype=torch.float64, device="cuda")
    dt_dev = torch.full((2,), dt, dtype=torch.float64, device="cuda")
    plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, nq, flags)
    try:
        torch.cuda.synchronize()
        fvpatch.fv_plan_capture_steps(plan, 1, a, c, h, wl.GAMMA, wl.CFL, lam, dt_dev, stream)
        paths = {
            "plain": lambda: fvpatch.fv_patch_batch_update(a, c, b.sizes, b.offsets, T, dim, nq, dt, h, wl.GAMMA,
                                                           flags, lam, stream=stream),
            "plain_contiguous": lambda: fvpatch.fv_patch_batch_update(a, c, b.sizes, None, T, dim, nq, dt, h,
                                                                      wl.GAMMA, flags, lam, stream=stream),
            "plan": lambda: fvpatch.fv_plan_execute(plan, a, c, dt, h, wl.GAMMA, lam, stream=stream),
            "graph": lambda: fvpatch.fv_plan_replay(plan, stream),
        }
        for path, call in paths.items():
            for _ in range(200):
                call()
            stream.synchronize()
            lat = np.empty(samples)
            for i in range(samples):
                t0 = time.perf_counter()
                call()
                stream.synchronize()
                lat[i] = time.perf_counter() - t0
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            n = 1000
            e0.record(stream)
            for _ in range(n):
                call()
            e1.record(stream)
            e1.synchronize()
            us = lat * 1e6
            line = {"metric": "launch-to-done latency", "form": "latency", "path": path,
                    "p50_us": round(float(np.percentile(us, 50)), 2), "p99_us": round(float(np.percentile(us, 99)), 2),
                    "max_us": round(float(us.max()), 2), "samples": samples, "unit": "us",
                    "device_us_per_launch_back_to_back": round(e0.elapsed_time(e1) * 1e3 / n, 2),
                    "cell_updates_per_call": int(b.interior_volumes()), "dtype": "f64", "data": "synthetic",
                    "higher_is_better": False,
                    "config": {"workload": name, "patches": T, "p": int(b.sizes[0]), "dim": dim, "unknowns": nq,
                               "state_bytes": int(b.data.nbytes)},
                    "timing": "host perf_counter from the call to hipStreamSynchronize's return, per sample"}
            print(json.dumps(line), flush=True)
    finally:
        fvpatch.fv_plan_destroy(plan)
    return 0


def bench_flavours(args) -> int:
    """The paper's matrix (p in {4, 6, 8}, d in {2, 3}, a sweep over T, with and without the
    eigenvalue reduction) for the fused update and the three comparison realisations
    (batched, patch-wise, task graph).  Time per step is wall time between device
    synchronisations over a few steps after two warmup steps, host work included: the task
    graph's per-call assembly is part of that realisation."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    flav = {"batched": fvpatch.FV_FLAVOUR_BATCHED, "patch_wise": fvpatch.FV_FLAVOUR_PATCH_WISE,
            "task_graph": fvpatch.FV_FLAVOUR_TASK_GRAPH}
    # 3D: only T = 16 -- the 3D sweep ended in a host segmentation fault at p = 4, T = 256 whose
    # cause is not identified, so larger 3D batches stay out of this comparison for now
    for dim, sweep in ((2, (16, 256, 4096, 65536)), (3, (16,))):
        for p in (4, 6, 8):
            base = wl.make_uniform(256, p, dim=dim, nq=5, seed=args.seed)
            for T in sweep:
                reps = (T + 255) // 256
                data = np.tile(base.data, reps)[: T * int(base.offsets[1])]
                sizes = np.full(T, p, np.int32)
                a = torch.from_numpy(data).to("cuda")
                c = a.clone()
                lam = torch.empty(T, dtype=torch.float64, device="cuda")
                for red in (True, False):
                    lam_arg = lam if red else None
                    line = {"form": "flavours", "dim": dim, "p": p, "patches": T, "reduction": red}

                    def timed(fn, steps):
                        bufs = [a, c]
                        for _ in range(2):
                            fn(bufs[0], bufs[1])
                            bufs.reverse()
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        for _ in range(steps):
                            fn(bufs[0], bufs[1])
                            bufs.reverse()
                        torch.cuda.synchronize()
                        return (time.perf_counter() - t0) / steps * 1e3

                    line["fused_ms"] = round(timed(lambda x, y: fvpatch.fv_patch_batch_update(
                        x, y, sizes, None, T, dim, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, 0, lam_arg), 10), 4)
                    for name, f in flav.items():
                        if name == "task_graph" and T > 4096:
                            line[name + "_ms"] = None
                            continue
                        steps = 3 if name == "task_graph" else 10
                        line[name + "_ms"] = round(timed(lambda x, y, f=f: fvpatch.fv_flavour_update(
                            f, x, y, sizes, None, T, dim, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, 0, lam_arg), steps), 4)
                    line["fused_cell_updates_per_s"] = round(T * p ** dim / (line["fused_ms"] / 1e3), 1)
                    print(json.dumps(line), flush=True)
                del a, c, lam
                torch.cuda.empty_cache()
    return 0


def bench_pde(args) -> int:
    """The generic solver of Eq. 1 (fv_pde_batch_update) on the shapes of the headline
    workloads: 2D shallow water (flux + non-conservative product + source, 4 unknowns with the
    bathymetry carried) and 2D acoustics in flux and non-conservative form on the 2D wave form
    (p = 16), 3D advection and acoustics on the 3D interior-mapped form (p = 8), and the Euler
    equations through the plane-marching kernel next to the tuned fixed-size kernel.  HIP events around the timed steps (ping-pong buffers, periodic face
    halos written, eigenvalue reduction on), per-step algorithmic bytes as in the headline."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    cases = [("shallow_water", 2, 16, 65536), ("acoustics", 2, 16, 65536), ("acoustics_ncp", 2, 16, 65536),
             ("euler", 2, 16, 65536), ("advection", 3, 8, 32768), ("acoustics", 3, 8, 32768),
             ("euler", 3, 8, 32768)]
    for name, dim, p, T in cases:
        b = wl.make_pde_batch(name, np.full(T, p), dim=dim, seed=args.seed)
        nq = b.nq
        prm = wl.default_params(name)
        a = torch.from_numpy(b.data).to("cuda")
        c = a.clone()
        lam = torch.empty(T, dtype=torch.float64, device="cuda")
        dt, h = 1e-4, wl.H_DEFAULT
        res = {}
        variants = [("generic", None)]
        if name == "euler":
            variants.append(("tuned", fvpatch.fv_get_tuning(dim, 5, p)))
        for label, tuned in variants:
            if name == "euler" and label == "generic":
                fvpatch.fv_set_tuning(dim, 5, p, {"kernel": fvpatch.FV_KERNEL_BLOCK})
            bufs = [a, c]

            def step():
                fvpatch.fv_pde_batch_update(fvpatch.PDE_IDS[name], prm, bufs[0], bufs[1], b.sizes, None, T, dim, dt,
                                            h, fvpatch.FV_HALO_PERIODIC, lam)
                bufs.reverse()

            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                step()
            e1.record()
            torch.cuda.synchronize()
            res[label] = e0.elapsed_time(e1) / args.steps
            if name == "euler" and label == "generic":
                fvpatch.fv_set_tuning(dim, 5, p, None)
        alg = T * alg_bytes_per_patch(p, dim, nq, True, True)
        ms = res["generic"]
        gbs = alg / (ms / 1e3) / 1e9
        line = {"metric": "cell-updates/s", "form": "pde", "pde": name, "value": round(T * p ** dim / (ms / 1e3), 1),
                "unit": "cell-updates/s", "ms_per_step": round(ms, 5), "alg_GBs": round(gbs, 1),
                "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_step": alg,
                "kernel": ("2D wave form (update2d_pde_kernel)" if dim == 2 and p in (3, 5, 9, 16, 17) and name != "euler"
                           else "3D interior-mapped form (update3d_pde_kernel)"
                           if dim == 3 and p in (4, 8) and name != "euler"
                           else "plane-marching kernel (update_kernel)"), "dtype": "f64", "data": "synthetic",
                "config": {"workload": f"{dim}D {name} {T} x {p}^{dim}", "patches": T, "p": p, "dim": dim,
                           "unknowns": nq, "params": prm, "periodic_halo": True, "eigenvalue_reduction": True,
                           "steps": args.steps}}
        if "tuned" in res:
            line["tuned_kernel_ms_per_step"] = round(res["tuned"], 5)
            line["generic_over_tuned"] = round(ms / res["tuned"], 3)
        print(json.dumps(line), flush=True)
        del a, c, lam
        torch.cuda.empty_cache()
    return 0


def bench_transfer(args) -> int:
    """Patches scattered in host memory (one allocation per patch, as on a mesh code's CPU
    heap) through one step on the GPU and back: per-patch synchronous copies into recycled
    device memory, the pipelined form (host threads each carrying chunks through gather into
    pinned staging, async copies, update, copy back and scatter, overlapped), and the staged
    form (threaded gather of the whole batch, one copy each way, no overlap), and zero copy (the
    same patches in pinned memory from fv_host_alloc, read and written over PCIe by gather /
    scatter kernels); against the device-resident step (no transfers) and the
    copy engines' own ceiling (pinned host <-> device copies of the same bytes, each
    direction alone and both at once).  Wall time per step between synchronisations."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    gamma, h, dt = wl.GAMMA, wl.H_DEFAULT, 1e-3
    for name in ("c2_2d_p16_T65536", "c4_3d_p8_T32768"):
        b, spec = wl.build_workload(name, seed=args.seed)
        T, p, dim, nq = b.num_patches, int(b.sizes[0]), b.dim, b.nq
        cells = T * p ** dim
        nbytes = b.data.nbytes
        src = wl.scatter_to_host(b, seed=args.seed)
        dst = [np.empty_like(a) for a in src]
        tin, tout = fvpatch.host_pointer_table(src), fvpatch.host_pointer_table(dst)
        lam = np.empty(T)

        def host_step(cfg, stats=None):
            fvpatch.fv_host_patches_update(tin, tout, b.sizes, T, dim, nq, dt, h, gamma, 0, lam, config=cfg,
                                           stats=stats)

        def wall(fn, warm, steps):
            """Median milliseconds of `steps` timed calls after `warm` untimed ones (each call
            is synchronous; the host's memory system makes single calls vary by ~10%)."""
            for _ in range(warm):
                fn()
            ts = []
            for _ in range(steps):
                t0 = time.perf_counter()
                fn()
                ts.append((time.perf_counter() - t0) * 1e3)
            return float(np.median(ts))

        res = {}
        # device-resident: the same step on patches already in HBM
        a = torch.from_numpy(b.data).to("cuda")
        c = a.clone()
        dlam = torch.empty(T, dtype=torch.float64, device="cuda")
        res["resident_ms"] = _timed_ms(lambda: fvpatch.fv_patch_batch_update(
            a, c, b.sizes, None, T, dim, nq, dt, h, gamma, 0, dlam), 10, 20)
        # copy-engine ceiling with pinned host memory
        hp_in = torch.empty(nbytes // 8, dtype=torch.float64, pin_memory=True)
        hp_out = torch.empty(nbytes // 8, dtype=torch.float64, pin_memory=True)
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

        def h2d():
            a.copy_(hp_in, non_blocking=True)

        def d2h():
            hp_out.copy_(c, non_blocking=True)

        def both():
            with torch.cuda.stream(s1):
                a.copy_(hp_in, non_blocking=True)
            with torch.cuda.stream(s2):
                hp_out.copy_(c, non_blocking=True)
            s1.synchronize()
            s2.synchronize()

        res["pinned_h2d_GBs"] = round(nbytes / _timed_ms(h2d, 2, 5) / 1e6, 2)
        res["pinned_d2h_GBs"] = round(nbytes / _timed_ms(d2h, 2, 5) / 1e6, 2)
        res["pinned_both_GBs"] = round(2 * nbytes / _timed_ms(both, 2, 5) / 1e6, 2)
        del hp_in, hp_out, a, c, dlam
        torch.cuda.empty_cache()
        # pipelined, defaults and a small sweep; staged without overlap; per patch
        stats = {}
        res["pipelined_ms"] = wall(lambda: host_step(None, stats), 3, 11)
        res["pipelined_host_copy_ms"] = stats["host_copy_seconds"] * 1e3
        sweep = []
        for chunk_mb, slots, threads in ((2, 2, 8), (4, 2, 8), (16, 2, 8), (32, 2, 8), (8, 1, 8), (8, 3, 8),
                                         (8, 2, 4), (8, 2, 12), (8, 2, 16)):
            cfg = {"chunk_bytes": chunk_mb << 20, "slots": slots, "host_threads": threads}
            sweep.append({"chunk_MiB": chunk_mb, "slots": slots, "host_threads": threads,
                          "ms": round(wall(lambda cfg=cfg: host_step(cfg), 1, 5), 3)})
        res["staged_no_overlap_ms"] = wall(lambda: host_step({"mode": fvpatch.FV_TRANSFER_STAGED}), 2, 7)
        pp_T = min(T, 8192)

        def per_patch():
            fvpatch.fv_host_patches_update(tin, tout, b.sizes, pp_T, dim, nq, dt, h, gamma, 0, lam,
                                           config={"mode": fvpatch.FV_TRANSFER_PER_PATCH})

        res["per_patch_ms_full_batch"] = wall(per_patch, 1, 2) * T / pp_T
        # zero copy: the same patches in pinned memory from fv_host_alloc (shuffled placement)
        a_in, a_out = fvpatch.fv_host_alloc(nbytes), fvpatch.fv_host_alloc(nbytes)
        try:
            big_in, big_out = fvpatch.pinned_array(a_in, nbytes // 8), fvpatch.pinned_array(a_out, nbytes // 8)
            n = nbytes // 8 // T
            place = np.random.Generator(np.random.PCG64(args.seed + 1)).permutation(T)
            zsrc = [big_in[place[t] * n:(place[t] + 1) * n] for t in range(T)]
            zdst = [big_out[place[t] * n:(place[t] + 1) * n] for t in range(T)]
            for t in range(T):
                zsrc[t][:] = src[t]
            zin, zout = fvpatch.host_pointer_table(zsrc), fvpatch.host_pointer_table(zdst)

            def zero_copy(cfg):
                fvpatch.fv_host_patches_update(zin, zout, b.sizes, T, dim, nq, dt, h, gamma, 0, lam,
                                               config=dict(cfg, mode=fvpatch.FV_TRANSFER_ZERO_COPY))

            res["zero_copy_ms"] = wall(lambda: zero_copy({}), 3, 11)
            zsweep = []
            for chunk_mb, slots in ((4, 2), (16, 2), (32, 2), (8, 4), (8, 8), (32, 4)):
                cfg = {"chunk_bytes": chunk_mb << 20, "slots": slots}
                zsweep.append({"chunk_MiB": chunk_mb, "slots": slots,
                               "ms": round(wall(lambda cfg=cfg: zero_copy(cfg), 1, 5), 3)})
            res["zero_copy_sweep"] = zsweep
            del zsrc, zdst, big_in, big_out
        finally:
            fvpatch.fv_host_free(a_in)
            fvpatch.fv_host_free(a_out)
        moved = 2 * nbytes + 8 * T
        ms = res["pipelined_ms"]
        line = {"metric": "cell-updates/s", "form": "transfer", "value": round(cells / (ms / 1e3), 1),
                "unit": "cell-updates/s", "ms_per_step": round(ms, 3),
                "transfer_GBs": round(moved / (ms / 1e3) / 1e9, 2),
                "frac_of_pinned_both": round(moved / (ms / 1e3) / 1e9 / res["pinned_both_GBs"], 3),
                "resident_ms_per_step": round(res["resident_ms"], 4),
                "staged_no_overlap_ms_per_step": round(res["staged_no_overlap_ms"], 3),
                "per_patch_ms_per_step": round(res["per_patch_ms_full_batch"], 1),
                "per_patch_measured_on": pp_T,
                "speedup_vs_per_patch": round(res["per_patch_ms_full_batch"] / ms, 2),
                "speedup_vs_staged": round(res["staged_no_overlap_ms"] / ms, 3),
                "host_copy_ms": round(res["pipelined_host_copy_ms"], 3),
                "pinned_h2d_GBs": res["pinned_h2d_GBs"], "pinned_d2h_GBs": res["pinned_d2h_GBs"],
                "pinned_both_GBs": res["pinned_both_GBs"], "sweep": sweep,
                "zero_copy_ms_per_step": round(res["zero_copy_ms"], 3),
                "zero_copy_GBs": round(moved / (res["zero_copy_ms"] / 1e3) / 1e9, 2),
                "zero_copy_sweep": res["zero_copy_sweep"],
                "dtype": "f64", "data": "synthetic",
                "config": {"workload": name, "patches": T, "p": p, "dim": dim,
                           "host_layout": "one allocation per patch, shuffled allocation order",
                           "bytes_each_way": nbytes},
                "timing": "median wall clock of synchronous calls (host gather / scatter and PCIe copies included)"}
        print(json.dumps(line), flush=True)
        del src, dst, tin, tout
    return 0


def _timed_ms(fn, warm: int, steps: int) -> float:
    """Milliseconds per call of fn over `steps` calls after `warm` untimed ones (device synchronised)."""
    import torch
    for _ in range(warm):
        fn()
    return _timed(fn, steps) / steps * 1e3


def bench_mesh(args) -> int:
    """Patch meshes with face halos from neighbours and local time stepping: the fused mesh
    step (fv_mesh_step: halos read from the neighbours in the kernel, per-patch dt / h) with
    per-patch step sizes formed on the device (fv_local_dt) after every step, against a
    separate halo fill followed by the plain launch (global dt) on the same mesh."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    steps, gamma = args.steps, wl.GAMMA
    for n, p, dim in ((256, 16, 2), (32, 8, 3)):
        m = wl.make_mesh(n, p, dim=dim, seed=args.seed, periodic=True)
        b = m.batch
        T, nq = b.num_patches, b.nq
        cells = T * p ** dim
        h = m.h
        a = torch.from_numpy(b.data).to("cuda")
        c = a.clone()
        lam = torch.empty(T, dtype=torch.float64, device="cuda")
        hv = torch.full((T,), h, dtype=torch.float64, device="cuda")
        mesh = fvpatch.fv_mesh_create(b.sizes, None, m.neighbors, T, dim, nq)
        try:
            # initial per-patch dt from the initial state's eigenvalues
            fvpatch.fv_mesh_step(mesh, a, c, torch.full((T,), 1e-9, dtype=torch.float64, device="cuda"), hv, gamma,
                                 lam)
            dt = torch.empty_like(lam)
            fvpatch.fv_local_dt(lam, hv, T, dim, wl.CFL, dt)
            dt0 = dt.clone()

            def fused_step(x, y):
                fvpatch.fv_mesh_step(mesh, x, y, dt, hv, gamma, lam)
                fvpatch.fv_local_dt(lam, hv, T, dim, wl.CFL, dt)

            dtg = float(dt0.min().item())

            def unfused_step(x, y):
                fvpatch.fv_mesh_halo_fill(mesh, x)
                fvpatch.fv_patch_batch_update(x, y, b.sizes, None, T, dim, nq, dtg, h, gamma, 0, lam)

            res = {}
            for name, fn in (("fused", fused_step), ("fill+plain", unfused_step)):
                bufs = [a, c]
                for _ in range(args.warmup):
                    fn(bufs[0], bufs[1])
                    bufs.reverse()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(steps):
                    fn(bufs[0], bufs[1])
                    bufs.reverse()
                e1.record()
                torch.cuda.synchronize()
                res[name] = e0.elapsed_time(e1) / steps
            dt_spread = (float(dt.min().item()), float(dt.max().item()))
        finally:
            fvpatch.fv_mesh_destroy(mesh)
        # the method's bytes: face-halo-padded input (halos are neighbours' interiors), interior output,
        # lambda, and the per-patch dt and h read / dt written
        alg = T * (((p ** dim + 2 * dim * p ** (dim - 1)) + p ** dim) * nq * 8 + 8 + 24)
        ms = res["fused"]
        line = {"metric": "cell-updates/s", "form": "mesh", "value": round(cells / (ms / 1e3), 1),
                "unit": "cell-updates/s", "ms_per_step": round(ms, 5), "alg_GBs": round(alg / (ms / 1e3) / 1e9, 1),
                "hbm_frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "fill_plus_plain_ms_per_step": round(res["fill+plain"], 5),
                "speedup_vs_fill_plus_plain": round(res["fill+plain"] / ms, 3),
                "local_dt_range": [round(v, 8) for v in dt_spread],
                "dtype": "f64", "data": "synthetic",
                "config": {"workload": f"{dim}D mesh {n}^{dim} x {p}^{dim}", "patches": T, "order": "Morton",
                           "halos": "face neighbours (periodic domain)", "time_stepping": "local (per-patch dt)",
                           "steps": steps},
                "timing": "HIP events around the timed steps (mesh step + per-patch dt)"}
        print(json.dumps(line), flush=True)
        del a, c
        torch.cuda.empty_cache()
    return 0


def bench_batching(args) -> int:
    """Configs 3 (200000 mixed 2D patches) and 4 (32768 x 8^3): plain per-batch launches vs a plan's fused
    launch vs the captured 10-step graph.  Wall time between device synchronisations (the plain path's host
    work counts: it is what the plan removes)."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import autotune, fvpatch
    from paper_2306_16731_amd import workloads as wl

    h, gamma, steps = wl.H_DEFAULT, wl.GAMMA, 10
    t_tune = time.perf_counter()
    if args.tuning_table:
        autotune.load(args.tuning_table)
        tuned = {"table": os.path.basename(args.tuning_table)}
    else:
        tuned = autotune.tune_classes([(2, 5, p) for p in (3, 5, 9, 17)] + [(3, 5, 8)], periodic=False)
    t_tune = time.perf_counter() - t_tune
    for name in ("c3_2d_mixed_T200000", "c4_3d_p8_T32768"):
        b, spec = wl.build_workload(name, seed=args.seed)
        T, dim, nq = b.num_patches, b.dim, b.nq
        periodic = spec["periodic"]
        flags = fvpatch.FV_HALO_PERIODIC if periodic else 0
        cells = b.interior_volumes()
        a = torch.from_numpy(b.data).to("cuda")
        c = a.clone()
        lam = torch.empty(T, dtype=torch.float64, device="cuda")
        dt = 1.0e-3
        bufs = [a, c]

        def plain():
            fvpatch.fv_patch_batch_update(bufs[0], bufs[1], b.sizes, b.offsets, T, dim, nq, dt, h, gamma, flags, lam)
            bufs.reverse()

        for _ in range(args.warmup // 10 + 3):
            plain()
        results = {"plain": _timed(plain, steps) / steps}
        plan_choice = autotune.tune_plan(b, periodic) if dim == 2 else {"mode": "persistent", "flags": 0}
        pflags = flags | plan_choice["flags"]
        plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, nq, pflags)
        try:
            info = fvpatch.fv_plan_info(plan)

            def fused():
                fvpatch.fv_plan_execute(plan, bufs[0], bufs[1], dt, h, gamma, lam)
                bufs.reverse()

            for _ in range(args.warmup // 10 + 3):
                fused()
            results["plan"] = _timed(fused, steps) / steps
            dt_dev = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
            stream = torch.cuda.Stream()
            fvpatch.fv_plan_capture_steps(plan, steps, a, c, h, gamma, wl.CFL, lam, dt_dev, stream)

            def replay():
                dt_dev[0] = dt
                fvpatch.fv_plan_replay(plan, stream)
                stream.synchronize()

            for _ in range(3):
                replay()
            results["graph"] = _timed(replay, 5) / (5 * steps)
            dts = dt_dev.cpu().numpy()
        finally:
            fvpatch.fv_plan_destroy(plan)
        if not periodic:
            # the same plan with the output's halo volumes given over (FV_HALO_FROM_IN): whole output rows
            plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, nq, pflags | fvpatch.FV_HALO_FROM_IN)
            try:
                def fused_whole():
                    fvpatch.fv_plan_execute(plan, bufs[0], bufs[1], dt, h, gamma, lam)
                    bufs.reverse()

                for _ in range(args.warmup // 10 + 3):
                    fused_whole()
                results["plan_halo_from_in"] = _timed(fused_whole, steps) / steps
            finally:
                fvpatch.fv_plan_destroy(plan)
        per_patch = [alg_bytes_per_patch(int(p), dim, nq, periodic, True) for p in b.sizes]
        alg = float(np.sum(per_patch))
        for form, sec in results.items():
            line = {"metric": "cell-updates/s", "value": round(cells / sec, 1), "unit": "cell-updates/s",
                    "form": form, "ms_per_step": round(sec * 1e3, 4), "alg_GBs": round(alg / sec / 1e9, 1),
                    "hbm_frac": round(alg / sec / 1e9 / HBM_PEAK_GBS, 4),
                    "speedup_vs_plain": round(results["plain"] / sec, 3), "dtype": "f64", "data": "synthetic",
                    "config": {"workload": name, "patches": T, "dim": dim, "steps": steps, "cells_per_step": cells,
                               "periodic_halo": periodic},
                    "plan": info if form != "plain" else None,
                    "plan_work_split": plan_choice if form != "plain" else None,
                    "timing": "wall time between device synchronisations, host work included"}
            if form == "graph":
                line["device_dt"] = [float(x) for x in dts[:3]]
            if form == "plan_halo_from_in":
                line["note"] = ("FV_HALO_FROM_IN: the output's halo volumes may take the input's values, so the "
                                "row-marching kernels write whole rows; algorithmic bytes counted without them")
            print(json.dumps(line), flush=True)
        del a, c, lam
        torch.cuda.empty_cache()
    print(json.dumps({"autotune_seconds": round(t_tune, 2), "tuning": tuned}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
