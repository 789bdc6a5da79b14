#!/usr/bin/env python3
"""Benchmark of the FV patch update on one MI355X.

Default workload: 65536 patches of 16 x 16 interior volumes (18 x 18 x 5
doubles each, AoS per volume), 2D compressible Euler, Rusanov flux, FP64,
seeded rho/u/v/w/p draws plus a Gaussian density pulse per patch, periodic
face-halo write and the per-patch eigenvalue reduction, as one
fv_patch_batch_update call per time step.  A "step" is one such call over the
whole batch (one explicit Euler time step of every patch).

Prints ONE JSON line with the metric (cell-updates/s, inputs resident in HBM),
the roofline of the update kernel (algorithmic bytes per launch / launch time,
against 8 TB/s), and the CPU oracle timed on a bounded sample of the same
workload on the host's cores.  Timing: W warmup steps, one K-step window
reported on its own (the first launches of a process run slower), untimed steps
up to 100 in all, then 16 windows of exactly K steps, each bracketed by device
synchronisations and timed by HIP events on the launch stream; the headline is
their median.  The same line carries config 1's launch-to-done latency and
configs 3 and 4 (plain launches, plan, captured graph) under "extra".

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]
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
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed steps first; the headline samples start after at least 100 steps in all")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-patches", type=int, default=65536,
                    help="at most this many patches for the CPU oracle (which advances them through the warmup "
                         "and the first timed window); the sample is sized to about 16 core-seconds")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the config-1 latency and config-3 / 4 batching keys")
    ap.add_argument("--form", choices=["plain", "batching", "serving", "mesh", "flavours", "transfer", "pde", "latency",
                                       "coldstart"],
                    default="plain",
                    help="plain: the headline line (config 2).  batching: configs 3 and 4 through plain launches, "
                         "plans and captured graphs (one line each).  serving: the request loop (config 5).  "
                         "latency: launch-to-done p50/p99 of config 1 (16 patches of 3^2, cache-resident)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the serving trace")
    ap.add_argument("--tuning-table", default=None, help="install this autotuner table instead of tuning now")
    ap.add_argument("--traffic-probe", nargs="?", const="c2", choices=["c2", "c3", "c4"], default=None,
                    help="run 4 launches of one workload's update (c2: the headline plain launch; c3: config 3's "
                         "fused plan launch, one wave per task; c4: config 4's plain launch, 3D 8^3, not periodic) "
                         "and one device copy of its state, for rocprofv3 --pmc runs (the copy's reading is the "
                         "counters' scale), then exit")
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
    if args.form == "coldstart":
        return bench_coldstart(args)
    if args.form == "serving":
        from paper_2306_16731_amd import serving
        return serving.bench_main(args)
    if args.traffic_probe in ("c3", "c4"):
        return traffic_probe(args)
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
    bufs = [d_a, d_b]

    def step():
        fvpatch.fv_patch_batch_update(bufs[0], bufs[1], b.sizes, None, T, dim, nq, dt, h, gamma, flags, lam, stream)
        bufs.reverse()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the first K-step window straight after the warmup, reported on its own: the first ~100
    # launches of a process run slower (bench.py --form coldstart measures why)
    t0 = time.perf_counter()
    first_ms = _window_ms(step, args.steps, stream)
    wall = time.perf_counter() - t0
    steps_done = args.warmup + args.steps
    # the oracle's sample is compared against the state after these warmup + K steps
    S = cpu_sample_patches(args, T, steps_done)
    sample_state = bufs[0][: S * int(b.offsets[1])].clone()
    settle = max(0, SETTLE_STEPS - steps_done)
    for _ in range(settle):
        step()
    # the headline: median of SAMPLES windows of exactly K steps, each bracketed by device
    # synchronisations and timed by HIP events on the launch stream
    samples = sorted(_window_ms(step, args.steps, stream) for _ in range(SAMPLES))
    ms_per_step = samples[len(samples) // 2]
    cells = T * p ** dim
    value = cells / (ms_per_step / 1e3)

    # a plain device copy of the state: the streaming ceiling of this GPU (sanity check of the roofline)
    scratch = torch.empty_like(d_a)
    for _ in range(3):
        scratch.copy_(d_a)
    copy_ms = _window_ms(lambda: scratch.copy_(d_a), 10, stream)
    copy_gbs = 2 * d_a.numel() * 8 / (copy_ms / 1e3) / 1e9
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
        "timing": {"headline": f"median of {SAMPLES} windows of {args.steps} steps, HIP events on the launch "
                               "stream, device synchronised around each window",
                   "settle_steps": settle, "samples_ms_per_step": [round(s, 5) for s in samples],
                   "first_window_ms_per_step": round(first_ms, 5),
                   "first_window_frac": round(per_launch / (first_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                   "first_window_host_wall_s": round(wall, 4)},
        "tuning": fvpatch.fv_get_tuning(dim, nq, p),
    }
    del bufs, d_a, d_b, lam
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        import oracle
        sub = b.data[: S * int(b.offsets[1])]
        threads = oracle.max_threads()
        t0 = time.perf_counter()
        ora_state, _ = oracle.run_steps(sub, b.sizes[:S], b.offsets[:S], dim, nq, [dt] * steps_done, h, gamma,
                                        periodic, nthreads=threads)
        cpu_s = time.perf_counter() - t0
        # one thread on a smaller sample of the same patches and steps
        S1 = max(1, S // 16)
        t1 = time.perf_counter()
        oracle.run_steps(b.data[: S1 * int(b.offsets[1])], b.sizes[:S1], b.offsets[:S1], dim, nq, [dt] * steps_done,
                         h, gamma, periodic, nthreads=1)
        cpu1_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(S * p ** dim * steps_done / cpu_s, 1), "unit": "cell-updates/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"first {S} of the {T} patches, {steps_done} steps, same dt, "
                                         f"OpenMP over patches ({cpu_s:.2f} s wall)",
                               "single_thread": {"value": round(S1 * p ** dim * steps_done / cpu1_s, 1),
                                                 "sample": f"first {S1} patches, {steps_done} steps "
                                                           f"({cpu1_s:.2f} s wall)"},
                               "cpu_work_core_s": round(cpu_s * threads + cpu1_s, 1),
                               "host_cpus_visible": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}
        # the GPU run advanced the same patches with the same dt: compare them
        got = sample_state.cpu().numpy()
        g = got.reshape(-1, nq)
        w = ora_state.reshape(-1, nq)
        errs = np.max(np.abs(g - w), axis=0) / np.max(np.abs(w), axis=0)
        out["parity_sample"] = {"patches": S, "steps": steps_done, "max_rel_err": float(np.max(errs)),
                                "tolerance": 1e-12}
    del sample_state
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["extra"] = extra_configs(args)
    print(json.dumps(out), flush=True)
    return 0


SETTLE_STEPS = 100  # untimed steps (warmup included) before the headline samples
SAMPLES = 16        # K-step windows whose median is the headline
CPU_TARGET_CORE_S = 16.0  # CPU work of the oracle's sample, in core-seconds
ORACLE_US_PER_PATCH_STEP = 40.0  # one core, one 16 x 16 patch, one step (measured on the host CPUs)


def traffic_probe(args) -> int:
    """--traffic-probe c3 / c4: four launches of the workload's update on its state, then one device copy of
    the state (bytes known), for rocprofv3 counter runs; prints one JSON line."""
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    name = {"c3": "c3_2d_mixed_T200000", "c4": "c4_3d_p8_T32768"}[args.traffic_probe]
    b, spec = wl.build_workload(name, seed=args.seed)
    T, dim, nq = b.num_patches, b.dim, b.nq
    flags = fvpatch.FV_HALO_PERIODIC if spec["periodic"] else 0
    a = torch.from_numpy(b.data).to("cuda")
    c = a.clone()
    lam = torch.empty(T, dtype=torch.float64, device="cuda")
    h, gamma, dt = wl.H_DEFAULT, wl.GAMMA, 1.0e-4
    plan = None
    if args.traffic_probe == "c3":
        plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, nq, flags | fvpatch.FV_PLAN_NO_PERSIST)
    try:
        for _ in range(4):
            if plan is not None:
                fvpatch.fv_plan_execute(plan, a, c, dt, h, gamma, lam)
            else:
                fvpatch.fv_patch_batch_update(a, c, b.sizes, b.offsets, T, dim, nq, dt, h, gamma, flags, lam)
        c.copy_(a)  # plain copy of known size: a.numel() * 8 bytes read and written
        torch.cuda.synchronize()
    finally:
        if plan is not None:
            fvpatch.fv_plan_destroy(plan)
    alg = int(sum(alg_bytes_per_patch(int(p), dim, nq, spec["periodic"], True) for p in b.sizes))
    print(json.dumps({"traffic_probe": args.traffic_probe, "workload": name, "copy_bytes": a.numel() * 8,
                      "alg_bytes_per_launch": alg, "kernel_sources_sha": kernel_sha()}))
    return 0


def cpu_sample_patches(args, T: int, steps: int) -> int:
    """Patches the oracle advances through all warmup + first-window steps: about
    CPU_TARGET_CORE_S core-seconds of work, a multiple of 256, at most --cpu-sample-patches."""
    s = int(CPU_TARGET_CORE_S / (ORACLE_US_PER_PATCH_STEP * 1e-6 * max(1, steps)))
    s = max(256, min(args.cpu_sample_patches, T, s))
    return s // 256 * 256


def _window_ms(fn, steps: int, stream) -> float:
    """Milliseconds per call over `steps` calls of fn: HIP events recorded on `stream` around
    them, the device synchronised before and after."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _median_window_ms(fn, steps: int, samples: int, stream) -> float:
    ts = sorted(_window_ms(fn, steps, stream) for _ in range(samples))
    return ts[len(ts) // 2]


def _settled_median_ms(fn, warmup: int, steps: int, samples: int = 5) -> float:
    """Milliseconds per call: at least SETTLE_STEPS untimed calls first (the first ~100 launches of a
    process run slower while the clocks ramp up), then the median of `samples` windows of `steps` calls,
    HIP events on the current stream."""
    import torch
    for _ in range(max(warmup, SETTLE_STEPS)):
        fn()
    return _median_window_ms(fn, steps, samples, torch.cuda.current_stream())


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
    launch and completion latency, not by HBM.  One JSON line per path (latency_lines)."""
    for line in latency_lines(args, samples):
        print(json.dumps(line), flush=True)
    return 0


def latency_lines(args, samples: int) -> list:
    """For the plain call, a plan's fused launch and a one-step captured graph: host time from the
    call to the stream's completion, per sample (p50 / p99 / max), and the device time per launch when
    launches run back to back.  The plain call runs twice: with an offsets array (evenly spaced, so
    nothing is uploaded) and contiguous (offsets NULL)."""
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
    torch.cuda.synchronize()
    plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, nq, flags)
    lines = []
    try:
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
            lines.append({"metric": "launch-to-done latency", "form": "latency", "path": path,
                          "p50_us": round(float(np.percentile(us, 50)), 2),
                          "p99_us": round(float(np.percentile(us, 99)), 2),
                          "max_us": round(float(us.max()), 2), "samples": samples, "unit": "us",
                          "device_us_per_launch_back_to_back": round(e0.elapsed_time(e1) * 1e3 / n, 2),
                          "cell_updates_per_call": int(b.interior_volumes()), "dtype": "f64", "data": "synthetic",
                          "higher_is_better": False,
                          "config": {"workload": name, "patches": T, "p": int(b.sizes[0]), "dim": dim,
                                     "unknowns": nq, "state_bytes": int(b.data.nbytes)},
                          "timing": "host perf_counter from the call to hipStreamSynchronize's return, per sample"})
    finally:
        fvpatch.fv_plan_destroy(plan)
    return lines


def extra_configs(args) -> dict:
    """The other configurations on the headline line: config 1's launch-to-done latency (p50 / p99)
    and configs 3 and 4 through plain launches, a plan and the captured 10-step graph (ms per step and
    fraction of the HBM roofline).  Class tunings are the library's defaults (every class of configs 3
    and 4 has a fixed-size build, which the fused launch runs whatever the tuning); config 3's plan
    launch mode is picked by timing the three modes (autotune.tune_plan)."""
    t0 = time.perf_counter()
    extra = {"c1_latency_us": {}}
    for line in latency_lines(args, 2000):
        extra["c1_latency_us"][line["path"]] = {k: line[k] for k in ("p50_us", "p99_us", "max_us")}
    for name in ("c3_2d_mixed_T200000", "c4_3d_p8_T32768"):
        r = batching_case(name, args, tune_plan_mode=True)
        e = {"cells_per_step": r["cells"], "alg_bytes_per_step": r["alg_bytes"], "plan_mode": r["plan_choice"]["mode"]}
        for form, ms in r["ms"].items():
            e[form + "_ms"] = round(ms, 4)
            e[form + "_frac"] = round(r["alg_bytes"] / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        e["speedup_plan_vs_plain"] = round(r["ms"]["plain"] / r["ms"]["plan"], 3)
        e["speedup_graph_vs_plain"] = round(r["ms"]["plain"] / r["ms"]["graph"], 3)
        extra[name] = e
    extra["timing"] = ("configs 3 / 4: median of 5 windows of 10 steps per form after at least 100 settle steps, "
                       "HIP events on one stream, "
                       "host launch work inside the window; graph: one 10-step replay per window")
    extra["seconds"] = round(time.perf_counter() - t0, 1)
    return extra


def bench_coldstart(args) -> int:
    """Where the slow first launches of a process come from.  Config 2's plain launch, one HIP event
    between consecutive launches, in three phases: (a) the first 150 launches of the process; (b) 50 more
    on the same buffers after the GPU sat idle for 2 s (if the clocks drop when idle, the slow start comes
    back here); (c) 50 on freshly allocated buffers while the GPU is busy and warm (new pages: if address
    translation is the cause, the slow start comes back here).  Prints one JSON line per phase with the
    per-launch times and their mean over launch windows."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import fvpatch
    from paper_2306_16731_amd import workloads as wl

    name = "c2_2d_p16_T65536"
    b, spec = wl.build_workload(name, seed=args.seed)
    T, dim, nq = b.num_patches, b.dim, b.nq
    flags = fvpatch.FV_HALO_PERIODIC
    h, gamma, dt = wl.H_DEFAULT, wl.GAMMA, 1.0e-3
    stream = torch.cuda.current_stream()
    per_launch = alg_bytes_per_patch(16, dim, nq, True, True) * T

    def run(a, c, n):
        lam = torch.empty(T, dtype=torch.float64, device="cuda")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        bufs = [a, c]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(n):
            fvpatch.fv_patch_batch_update(bufs[0], bufs[1], b.sizes, None, T, dim, nq, dt, h, gamma, flags, lam,
                                          stream)
            bufs.reverse()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(n)])

    a = torch.from_numpy(b.data).to("cuda")
    c = a.clone()
    phases = {"a_fresh_process": run(a, c, 150)}
    time.sleep(2.0)
    phases["b_after_2s_idle_same_buffers"] = run(a, c, 50)
    a2 = torch.empty_like(a)
    c2 = torch.empty_like(c)
    a2.copy_(a)  # warm GPU; a2's pages are new to the update kernel (the copy touched them once)
    phases["c_fresh_buffers_warm_gpu"] = run(a2, c2, 50)
    for phase, ms in phases.items():
        win = [round(float(ms[i:i + 10].mean()), 4) for i in range(0, len(ms), 10)]
        print(json.dumps({"form": "coldstart", "phase": phase, "launches": len(ms),
                          "mean_ms_per_10_launches": win, "first_ms": round(float(ms[0]), 4),
                          "last10_mean_ms": round(float(ms[-10:].mean()), 4),
                          "first10_frac": round(per_launch / (float(ms[:10].mean()) / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                          "last10_frac": round(per_launch / (float(ms[-10:].mean()) / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                          "per_launch_ms": [round(float(x), 4) for x in ms],
                          "config": {"workload": name}}), flush=True)
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
    for dim, sweep in ((2, (16, 256, 4096, 65536)), (3, (16, 256, 4096, 32768))):
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
    equations through the plane-marching kernel next to the tuned fixed-size kernel.  Median of 5 windows of
    the timed steps after >= 100 settle steps, HIP events (ping-pong buffers, periodic face
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

            res[label] = _settled_median_ms(step, args.warmup, args.steps)
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

                def step(fn=fn, bufs=bufs):
                    fn(bufs[0], bufs[1])
                    bufs.reverse()

                res[name] = _settled_median_ms(step, args.warmup, steps)
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
                "timing": "median of 5 windows of the timed steps after >= 100 settle steps, HIP events (mesh step + "
                          "per-patch dt)"}
        print(json.dumps(line), flush=True)
        del a, c
        torch.cuda.empty_cache()
    return 0


def batching_case(name: str, args, tune_plan_mode: bool, steps: int = 10, samples: int = 5, tune=None) -> dict:
    """One batching workload (config 3 or 4) through plain per-batch launches, a plan's fused launch,
    the plan's captured `steps`-step graph with device dt and, when the workload is not periodic, the
    plan with FV_HALO_FROM_IN.  ms per step: median of `samples` windows of `steps` steps after at least
    SETTLE_STEPS untimed steps of the same form (a GPU left idle by the host work between forms starts
    slow), HIP events on one stream (the plain path's host work, which the plan removes, is inside the
    window)."""
    import numpy as np
    import torch

    from paper_2306_16731_amd import autotune, fvpatch
    from paper_2306_16731_amd import workloads as wl

    h, gamma = wl.H_DEFAULT, wl.GAMMA
    b, spec = wl.build_workload(name, seed=args.seed)
    T, dim, nq = b.num_patches, b.dim, b.nq
    periodic = spec["periodic"]
    flags = fvpatch.FV_HALO_PERIODIC if periodic else 0
    if dim == 2 and tune_plan_mode:
        plan_choice = autotune.tune_plan(b, periodic, tune=tune)
    elif dim == 2:
        plan_choice = {"mode": "per_task", "flags": fvpatch.FV_PLAN_NO_PERSIST}
    else:
        plan_choice = {"mode": "persistent", "flags": 0}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = torch.from_numpy(b.data).to("cuda")
        c = a.clone()
        lam = torch.empty(T, dtype=torch.float64, device="cuda")
        dt_dev = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    dt = 1.0e-3
    bufs = [a, c]
    ms = {}

    def plain():
        fvpatch.fv_patch_batch_update(bufs[0], bufs[1], b.sizes, b.offsets, T, dim, nq, dt, h, gamma, flags, lam,
                                      stream=s)
        bufs.reverse()

    settle = max(3, SETTLE_STEPS)  # untimed steps before each form's windows (clocks settle)
    for _ in range(settle):
        plain()
    ms["plain"] = _median_window_ms(plain, steps, samples, s)
    pflags = flags | plan_choice["flags"]
    plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, nq, pflags, tune=tune)
    try:
        info = fvpatch.fv_plan_info(plan)

        def fused():
            fvpatch.fv_plan_execute(plan, bufs[0], bufs[1], dt, h, gamma, lam, stream=s)
            bufs.reverse()

        for _ in range(settle):
            fused()
        ms["plan"] = _median_window_ms(fused, steps, samples, s)
        fvpatch.fv_plan_capture_steps(plan, steps, a, c, h, gamma, wl.CFL, lam, dt_dev, s)

        def replay():
            with torch.cuda.stream(s):
                dt_dev[0] = dt
            fvpatch.fv_plan_replay(plan, s)

        for _ in range(max(2, settle // steps)):
            replay()
        ms["graph"] = _median_window_ms(replay, 1, samples, s) / steps
        dts = dt_dev.cpu().numpy()
    finally:
        fvpatch.fv_plan_destroy(plan)
    if not periodic:
        plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, nq, pflags | fvpatch.FV_HALO_FROM_IN, tune=tune)
        try:
            def fused_whole():
                fvpatch.fv_plan_execute(plan, bufs[0], bufs[1], dt, h, gamma, lam, stream=s)
                bufs.reverse()

            for _ in range(settle):
                fused_whole()
            ms["plan_halo_from_in"] = _median_window_ms(fused_whole, steps, samples, s)
            fvpatch.fv_plan_capture_steps(plan, steps, a, c, h, gamma, wl.CFL, lam, dt_dev, s)

            def replay_whole():
                with torch.cuda.stream(s):
                    dt_dev[0] = dt
                fvpatch.fv_plan_replay(plan, s)

            for _ in range(max(2, settle // steps)):
                replay_whole()
            ms["graph_halo_from_in"] = _median_window_ms(replay_whole, 1, samples, s) / steps
        finally:
            fvpatch.fv_plan_destroy(plan)
    alg = float(np.sum([alg_bytes_per_patch(int(p), dim, nq, periodic, True) for p in b.sizes]))
    del a, c, lam, bufs, dt_dev
    torch.cuda.empty_cache()
    return {"name": name, "ms": ms, "alg_bytes": alg, "cells": b.interior_volumes(), "T": T, "dim": dim,
            "periodic": periodic, "plan_info": info, "plan_choice": plan_choice, "device_dt": [float(x) for x in dts[:3]],
            "steps": steps}


def bench_batching(args) -> int:
    """Configs 3 (200000 mixed 2D patches) and 4 (32768 x 8^3): plain per-batch launches vs a plan's fused
    launch vs the captured 10-step graph, after the autotuner has set every class (or a table is loaded)."""
    from paper_2306_16731_amd import autotune

    t_tune = time.perf_counter()
    if args.tuning_table:
        entries = autotune.load(args.tuning_table)["entries"]
        tuned = {"table": os.path.basename(args.tuning_table)}
    else:
        # installed process-wide for the plain launches; the plans get the same table as their own
        entries = tuned = autotune.tune_classes([(2, 5, p) for p in (3, 5, 9, 17)] + [(3, 5, 8)], periodic=False)
    table = autotune.plan_table(entries)
    t_tune = time.perf_counter() - t_tune
    for name in ("c3_2d_mixed_T200000", "c4_3d_p8_T32768"):
        r = batching_case(name, args, tune_plan_mode=True, tune=table)
        for form, ms in r["ms"].items():
            sec = ms / 1e3
            line = {"metric": "cell-updates/s", "value": round(r["cells"] / sec, 1), "unit": "cell-updates/s",
                    "form": form, "ms_per_step": round(ms, 4), "alg_GBs": round(r["alg_bytes"] / sec / 1e9, 1),
                    "hbm_frac": round(r["alg_bytes"] / sec / 1e9 / HBM_PEAK_GBS, 4),
                    "speedup_vs_plain": round(r["ms"]["plain"] / ms, 3), "dtype": "f64", "data": "synthetic",
                    "config": {"workload": name, "patches": r["T"], "dim": r["dim"], "steps": r["steps"],
                               "cells_per_step": r["cells"], "periodic_halo": r["periodic"]},
                    "plan": r["plan_info"] if form != "plain" else None,
                    "plan_work_split": r["plan_choice"] if form != "plain" else None,
                    "timing": "median of 5 windows of 10 steps after at least 100 settle steps, HIP events on one "
                              "stream, host work included"}
            if form == "graph":
                line["device_dt"] = r["device_dt"]
            if form in ("plan_halo_from_in", "graph_halo_from_in"):
                line["note"] = ("FV_HALO_FROM_IN: the output's halo volumes may take the input's values, so the "
                                "row-marching kernels write whole rows; algorithmic bytes counted without them")
            print(json.dumps(line), flush=True)
    print(json.dumps({"autotune_seconds": round(t_tune, 2), "tuning": tuned}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
