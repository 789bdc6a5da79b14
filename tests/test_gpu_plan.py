"""Batching form (plans) vs the CPU oracle through the C ABI (needs a gfx950 GPU).

A plan runs every size class of a mixed batch in one fused launch (persistent
or one wave per task) or in one launch per class, per-class launches for 3D and
2D p > 62 in every mode, and captures k
steps with a device-side time step in a hipGraph.  Tolerance as for the plain
launch: 1e-12 per-unknown relative max-norm, and the same for lambda and for the
device-formed time steps.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2306_16731_amd import workloads as wl
from tests import hip_path as hp

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _announce(msg):
    print(f"[gpu-plan] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16731_amd import fvpatch
    fvpatch.load()


def oracle_dts(batch, steps, periodic, dt0, h=wl.H_DEFAULT, cfl=wl.CFL):
    """The step sizes the oracle's own eigenvalues give, starting from dt0."""
    state = batch.data.copy()
    dts = [dt0]
    for _ in range(steps):
        state, lam = oracle.batch_update(state, batch.sizes, batch.offsets, batch.dim, batch.nq, dts[-1], h,
                                         wl.GAMMA, periodic)
        dts.append(cfl * h / (batch.dim * float(np.max(lam))))
    return dts


def run_plan(batch, dts, periodic, flags=0, tune=None):
    import torch
    from paper_2306_16731_amd import fvpatch
    plan = fvpatch.fv_plan_create(batch.sizes, batch.offsets, batch.num_patches, batch.dim, batch.nq,
                                  flags | (fvpatch.FV_HALO_PERIODIC if periodic else 0), tune=tune)
    try:
        info = fvpatch.fv_plan_info(plan)
        a = hp.to_dev(batch.data)
        b = a.clone()
        lam = torch.empty((len(dts), batch.num_patches), dtype=torch.float64, device="cuda")
        for s, dt in enumerate(dts):
            fvpatch.fv_plan_execute(plan, a, b, dt, wl.H_DEFAULT, wl.GAMMA, lam[s])
            a, b = b, a
        torch.cuda.synchronize()
        return a.cpu().numpy(), list(lam.cpu().numpy()), info
    finally:
        fvpatch.fv_plan_destroy(plan)


def check_against_oracle(batch, dts, periodic, got, got_lams):
    want, want_lams = oracle.run_steps(batch.data, batch.sizes, batch.offsets, batch.dim, batch.nq, dts,
                                       wl.H_DEFAULT, wl.GAMMA, periodic)
    errs = hp.component_errors(got, want, batch.nq)
    assert np.all(errs <= TOL), errs
    assert max(hp.lambda_error(g, w) for g, w in zip(got_lams, want_lams)) <= TOL


@pytest.mark.parametrize("mode", ["persistent", "per_task", "per_class"])
def test_plan_mixed_sizes(mode):
    from paper_2306_16731_amd import fvpatch
    _announce(f"plan: 3000 mixed {{3,5,9,17}}^2, 6 steps, mode={mode}")
    b, _ = wl.build_workload("c3_2d_mixed_T200000", seed=21, num_patches=3000)
    dts = oracle_dts(b, 5, False, 1.5e-3)
    flags = {"persistent": 0, "per_task": fvpatch.FV_PLAN_NO_PERSIST, "per_class": fvpatch.FV_PLAN_PER_CLASS}[mode]
    got, lams, info = run_plan(b, dts, False, flags)
    if mode == "per_class":
        assert info["num_class_launches"] == 4 and info["num_tasks"] == 0
    else:
        assert info["num_class_launches"] == 0 and info["num_tasks"] > 0
        assert info["persistent"] == int(mode == "persistent")
    check_against_oracle(b, dts, False, got, lams)


@pytest.mark.parametrize("periodic,from_in", [(False, False), (True, False), (False, True)])
def test_plan_modes_agree_bitwise(periodic, from_in):
    """The fused launch and the per-class launches run the same fixed-size bodies in the same
    order of operations, whatever their load and store widths, ring depths and rows in flight:
    outputs and eigenvalues agree bit for bit with each other and with the plain per-batch launch,
    on gapped offsets.  With FV_HALO_FROM_IN the output halos take the input's, which are the
    initial halos in both buffers here, so the state still equals the oracle's."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"plan modes bitwise, periodic={periodic}, from_in={from_in}")
    extra = fvpatch.FV_HALO_FROM_IN if from_in else 0
    rng = np.random.Generator(np.random.PCG64(41))
    sizes = rng.choice(np.array([3, 5, 9, 16, 17, 30], np.int32), size=700)
    compact = wl.make_batch(sizes, 2, 5, seed=42)
    vols = (sizes.astype(np.int64) + 2) ** 2 * 5
    # every patch starts at an even double (16-byte loads and stores for the even-sized classes
    # p = 16, 30), or, periodic case, from the first p = 16 patch on at shifted parity
    gaps = rng.integers(0, 3, size=len(sizes)) * 2 + vols % 2
    if periodic:
        gaps[int(np.argmax(sizes == 16))] += 1
    starts = np.cumsum(np.concatenate([[0], (vols + gaps)[:-1]])).astype(np.int64)
    data = np.zeros(int(starts[-1] + vols[-1] + 2))
    for t in range(len(sizes)):
        data[starts[t]:starts[t] + vols[t]] = compact.data[compact.offsets[t]:compact.offsets[t] + vols[t]]
    batch = wl.Batch(data=data, sizes=sizes, offsets=starts, dim=2, nq=5)
    dts = [1.1e-3, 0.9e-3]
    results = {}
    for mode, flags in [("persistent", 0), ("per_task", fvpatch.FV_PLAN_NO_PERSIST),
                        ("per_class", fvpatch.FV_PLAN_PER_CLASS)]:
        got, lams, info = run_plan(batch, dts, periodic, flags | extra)
        results[mode] = (got, np.stack(lams))
    fl = (fvpatch.FV_HALO_PERIODIC if periodic else 0) | extra
    a = hp.to_dev(data)
    b2 = a.clone()
    lam = torch.empty((len(dts), len(sizes)), dtype=torch.float64, device="cuda")
    for s, dt in enumerate(dts):
        fvpatch.fv_patch_batch_update(a, b2, sizes, starts, len(sizes), 2, 5, dt, wl.H_DEFAULT, wl.GAMMA, fl, lam[s])
        a, b2 = b2, a
    torch.cuda.synchronize()
    results["plain"] = (a.cpu().numpy(), lam.cpu().numpy())
    ref = results["per_class"]
    for mode, (got, lams) in results.items():
        assert np.array_equal(got, ref[0]) and np.array_equal(lams, ref[1]), mode
    mask = np.zeros(len(data), bool)
    for t in range(len(sizes)):
        mask[starts[t]:starts[t] + vols[t]] = True
    assert np.array_equal(ref[0][~mask], data[~mask])
    want, want_lams = oracle.run_steps(data, sizes, starts, 2, 5, dts, wl.H_DEFAULT, wl.GAMMA, periodic)
    assert np.all(hp.component_errors(ref[0][mask], want[mask], 5) <= TOL)
    assert max(hp.lambda_error(g, w) for g, w in zip(ref[1], want_lams)) <= TOL


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("persistent", [True, False])
def test_plan_mixed_sizes_runtime_size_bodies(periodic, persistent):
    """The task list with runtime-size bodies (sizes without a fixed-size build, tuned rows and
    prefetch) beside fixed-size ones, so both task bodies stay covered in both task orders."""
    from paper_2306_16731_amd import fvpatch
    _announce(f"plan: mixed sizes, runtime-size bodies, periodic={periodic}, persistent={persistent}")
    b = wl.make_mixed(1500, choices=(4, 7, 12, 20, 9), seed=24)
    table = {(2, 5, p): dict(kernel=fvpatch.FV_KERNEL_WAVE, block=256, prefetch=3, rows=4) for p in (4, 7, 12, 20)}
    dts = oracle_dts(b, 3, periodic, 1.5e-3)
    got, lams, info = run_plan(b, dts, periodic, 0 if persistent else fvpatch.FV_PLAN_NO_PERSIST, tune=table)
    assert info["prefetch"] == 3
    check_against_oracle(b, dts, periodic, got, lams)


def test_two_plans_with_their_own_tuning_tables_side_by_side():
    """Two plans over the same mixed batch, each launching every class on its own kernel with its own
    table (tile / block / wave kernels with different blocks and rows per class), stepped alternately
    in one process: each reports its own resolved tuning, the process-wide tuning is untouched, and
    both match the oracle (and each other, bit for bit: every kernel rounds the same way)."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce("two plans, two tuning tables")
    K = fvpatch
    b = wl.make_mixed(900, choices=(4, 7, 12, 9), seed=25)
    tables = {
        "a": {(2, 5, 4): dict(kernel=K.FV_KERNEL_TILE, block=64), (2, 5, 7): dict(kernel=K.FV_KERNEL_BLOCK, block=128),
              (2, 5, 12): dict(kernel=K.FV_KERNEL_WAVE, block=128, prefetch=2, rows=8),
              (3, 5, 8): dict(kernel=K.FV_KERNEL_BLOCK, block=128)},   # another dim: ignored
        "b": {(2, 5, 4): dict(kernel=K.FV_KERNEL_WAVE, block=256, prefetch=4, rows=4),
              (2, 5, 7): dict(kernel=K.FV_KERNEL_WAVE, block=128, prefetch=2, rows=6),
              (2, 5, 12): dict(kernel=K.FV_KERNEL_BLOCK, block=256), (2, 5, 9): dict(kernel=K.FV_KERNEL_TILE)},
    }
    before = {p: K.fv_get_tuning(2, 5, p) for p in (4, 7, 9, 12)}
    flags = K.FV_PLAN_PER_CLASS | K.FV_HALO_PERIODIC
    plans = {k: K.fv_plan_create(b.sizes, b.offsets, b.num_patches, 2, 5, flags, tune=t) for k, t in tables.items()}
    try:
        assert {p: K.fv_get_tuning(2, 5, p) for p in (4, 7, 9, 12)} == before
        assert K.fv_plan_get_tuning(plans["a"], 4)["kernel"] == K.FV_KERNEL_TILE
        assert K.fv_plan_get_tuning(plans["b"], 4)["kernel"] == K.FV_KERNEL_WAVE
        assert K.fv_plan_get_tuning(plans["a"], 12) == dict(kernel=K.FV_KERNEL_WAVE, block=128, prefetch=2, rows=8)
        assert K.fv_plan_get_tuning(plans["b"], 12)["kernel"] == K.FV_KERNEL_BLOCK
        assert K.fv_plan_get_tuning(plans["a"], 9) == before[9]     # no entry: the installed default
        assert K.fv_plan_get_tuning(plans["b"], 9)["kernel"] == K.FV_KERNEL_TILE
        dts = oracle_dts(b, 3, True, 1.2e-3)
        bufs = {k: [hp.to_dev(b.data), None] for k in plans}
        for k in bufs:
            bufs[k][1] = bufs[k][0].clone()
        lams = {k: torch.empty((len(dts), b.num_patches), dtype=torch.float64, device="cuda") for k in plans}
        for step, dt in enumerate(dts):
            for k, plan in plans.items():      # alternate between the plans every step
                K.fv_plan_execute(plan, bufs[k][0], bufs[k][1], dt, wl.H_DEFAULT, wl.GAMMA, lams[k][step])
                bufs[k].reverse()
        torch.cuda.synchronize()
        got = {k: (bufs[k][0].cpu().numpy(), list(lams[k].cpu().numpy())) for k in plans}
    finally:
        for plan in plans.values():
            K.fv_plan_destroy(plan)
    assert np.array_equal(got["a"][0], got["b"][0])
    for k in plans:
        check_against_oracle(b, dts, True, *got[k])


@pytest.mark.parametrize("name,T", [("c3_2d_mixed_T200000", 1200), ("c4_3d_p8_T32768", 100)])
def test_plan_execute_with_device_dt(name, T):
    """fv_plan_execute with dt in device memory: the step reads it when it runs, and the result equals
    the host-dt step bit for bit (dt / h is correctly rounded on both sides)."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"plan execute with device dt: {name} T={T}")
    b, _ = wl.build_workload(name, seed=26, num_patches=T)
    plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, b.dim, b.nq, fvpatch.FV_PLAN_NO_PERSIST if b.dim == 2 else 0)
    try:
        dts = [1.3e-3, 0.7e-3, 1.1e-3]
        res = {}
        for mode in ("host", "device"):
            a = hp.to_dev(b.data)
            c = a.clone()
            lam = torch.empty((len(dts), T), dtype=torch.float64, device="cuda")
            dt_dev = torch.full((1,), 99.0, dtype=torch.float64, device="cuda")
            for k, dt in enumerate(dts):
                if mode == "host":
                    fvpatch.fv_plan_execute(plan, a, c, dt, wl.H_DEFAULT, wl.GAMMA, lam[k])
                else:
                    dt_dev.fill_(dt)     # ordered before the step on the same stream
                    fvpatch.fv_plan_execute(plan, a, c, -1.0, wl.H_DEFAULT, wl.GAMMA, lam[k], dt_dev=dt_dev)
                a, c = c, a
            torch.cuda.synchronize()
            res[mode] = (a.cpu().numpy(), lam.cpu().numpy())
        d = hp.to_dev(b.data)
        out = d.clone()
        assert fvpatch.fv_plan_execute(plan, d, out, 1e-3, wl.H_DEFAULT, wl.GAMMA, None, dt_dev=out[3:4],
                                       raise_on_error=False) == fvpatch.FV_ERR_OVERLAP
    finally:
        fvpatch.fv_plan_destroy(plan)
    assert np.array_equal(res["host"][0], res["device"][0])
    assert np.array_equal(res["host"][1], res["device"][1])
    check_against_oracle(b, dts, False, res["device"][0], list(res["device"][1]))


def test_plan_mixed_with_large_class_odd_offsets_periodic():
    """Sizes the wave kernel cannot take (p = 63, 64) run as class launches in the same step;
    patches start at odd doubles (8- not 16-byte aligned), with gaps."""
    _announce("plan: mixed with p in {1, 7, 16, 63, 64}, odd offsets, periodic")
    rng = np.random.Generator(np.random.PCG64(31))
    sizes = rng.choice(np.array([1, 7, 16, 63, 64], np.int32), size=150)
    compact = wl.make_batch(sizes, 2, 5, seed=32)
    vols = (sizes.astype(np.int64) + 2) ** 2 * 5
    starts = np.cumsum(np.concatenate([[1], (vols + 3)[:-1]])).astype(np.int64)
    data = np.zeros(int(starts[-1] + vols[-1] + 1))
    for t in range(len(sizes)):
        data[starts[t]:starts[t] + vols[t]] = compact.data[compact.offsets[t]:compact.offsets[t] + vols[t]]
    batch = wl.Batch(data=data, sizes=sizes, offsets=starts, dim=2, nq=5)
    dts = [1.1e-3, 0.9e-3, 1.2e-3]
    got, lams, info = run_plan(batch, dts, True)
    assert info["num_class_launches"] == 2
    mask = np.zeros(len(data), bool)
    for t in range(len(sizes)):
        mask[starts[t]:starts[t] + vols[t]] = True
    assert np.array_equal(got[~mask], data[~mask])
    want, want_lams = oracle.run_steps(data, sizes, starts, 2, 5, dts, wl.H_DEFAULT, wl.GAMMA, True)
    assert np.all(hp.component_errors(got[mask], want[mask], 5) <= TOL)
    assert max(hp.lambda_error(g, w) for g, w in zip(lams, want_lams)) <= TOL


def test_plan_3d():
    _announce("plan: 300 x 8^3, 4 steps")
    b, _ = wl.build_workload("c4_3d_p8_T32768", seed=22, num_patches=300)
    dts = oracle_dts(b, 3, False, 1.2e-3)
    got, lams, info = run_plan(b, dts, False)
    assert info["num_tasks"] == 0 and info["num_class_launches"] == 1
    check_against_oracle(b, dts, False, got, lams)


@pytest.mark.parametrize("name,T,periodic,per_class,from_in", [("c3_2d_mixed_T200000", 2500, False, False, False),
                                                               ("c3_2d_mixed_T200000", 2500, True, True, False),
                                                               ("c3_2d_mixed_T200000", 2500, False, False, True),
                                                               ("c4_3d_p8_T32768", 200, False, False, False),
                                                               ("c4_3d_p8_T32768", 200, False, False, True),
                                                               ("c2_2d_p16_T65536", 600, True, False, False)])
def test_graph_replay_with_device_dt(name, T, periodic, per_class, from_in):
    """k steps captured in one graph; step sizes formed on the device from each step's
    eigenvalues.  Replayed twice with eager work and synchronisations in between;
    every replay is checked against the oracle run with the device's step sizes,
    and those step sizes against the ones the oracle's own eigenvalues give.  With
    FV_HALO_FROM_IN the output halos take the input's values, which here are the initial
    halos in both buffers, so the whole state still equals the oracle's."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"graph: {name} T={T}, periodic={periodic}, per_class={per_class}, from_in={from_in}, "
              "5 steps x 2 replays")
    b, _ = wl.build_workload(name, seed=23, num_patches=T)
    steps = 5
    plan = fvpatch.fv_plan_create(b.sizes, b.offsets, b.num_patches, b.dim, b.nq,
                                  (fvpatch.FV_HALO_PERIODIC if periodic else 0) |
                                  (fvpatch.FV_PLAN_PER_CLASS if per_class else 0) |
                                  (fvpatch.FV_HALO_FROM_IN if from_in else 0))
    try:
        bufa = hp.to_dev(b.data)
        bufb = bufa.clone()
        lam = torch.empty(b.num_patches, dtype=torch.float64, device="cuda")
        dt_dev = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        fvpatch.fv_plan_capture_steps(plan, steps, bufa, bufb, wl.H_DEFAULT, wl.GAMMA, wl.CFL, lam, dt_dev, s)
        assert fvpatch.fv_plan_info(plan)["captured_steps"] == steps
        state = b.data.copy()
        dt0 = 1.4e-3
        for rep in range(2):
            dt_dev[0] = dt0
            torch.cuda.synchronize()
            fvpatch.fv_plan_replay(plan, s)
            s.synchronize()
            got = (bufb if steps % 2 else bufa).cpu().numpy()
            dts = dt_dev.cpu().numpy()
            # eager work between replays (torch kernels, a copy, a sync)
            scratch = torch.ones(1 << 20, device="cuda").cumsum(0)
            torch.cuda.synchronize()
            del scratch
            want, want_lams = oracle.run_steps(state, b.sizes, b.offsets, b.dim, b.nq, list(dts[:steps]),
                                               wl.H_DEFAULT, wl.GAMMA, periodic)
            assert np.all(hp.component_errors(got, want, b.nq) <= TOL), rep
            assert hp.lambda_error(lam.cpu().numpy(), want_lams[-1]) <= TOL
            ref_dts = [dts[0]] + [wl.CFL * wl.H_DEFAULT / (b.dim * float(np.max(l))) for l in want_lams]
            np.testing.assert_allclose(dts, ref_dts, rtol=TOL, atol=0)
            # the next replay starts from this result: bring it back into buffer a
            if steps % 2:
                bufa.copy_(bufb)
            torch.cuda.synchronize()
            state = want
            dt0 = float(dts[-1])
    finally:
        fvpatch.fv_plan_destroy(plan)


@pytest.mark.parametrize("dim,p,gap,per_class,flags", [(2, 17, 3, True, "periodic"), (2, 16, 0, True, "none"),
                                                      (3, 8, 0, False, "none"), (3, 4, 2, False, "from_in"),
                                                      (3, 6, 1, False, "periodic")])
def test_plan_regular_class_launches_without_descriptors(dim, p, gap, per_class, flags):
    """A class whose patches are evenly spaced, in order, launches like a plain call on such a batch (no
    descriptors): the plan's steps equal the plain per-batch launch's bit for bit, at any spacing, and
    the bytes between patches stay untouched."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"plan: regular class dim={dim} p={p} gap={gap} per_class={per_class} flags={flags}")
    T = 700 if dim == 2 else 300
    compact = wl.make_uniform(T, p, dim=dim, nq=5, seed=51)
    vol = (p + 2) ** dim * 5
    offsets = 1 + np.arange(T, dtype=np.int64) * (vol + gap)
    data = np.random.Generator(np.random.PCG64(52)).uniform(-1, 1, int(offsets[-1] + vol + 2))
    for t in range(T):
        data[offsets[t]:offsets[t] + vol] = compact.data[compact.offsets[t]:compact.offsets[t] + vol]
    fl = {"none": 0, "periodic": fvpatch.FV_HALO_PERIODIC, "from_in": fvpatch.FV_HALO_FROM_IN}[flags]
    sizes = np.full(T, p, np.int32)
    dts = [1.2e-3, 0.8e-3]
    res = {}
    plan = fvpatch.fv_plan_create(sizes, offsets, T, dim, 5, fl | (fvpatch.FV_PLAN_PER_CLASS if per_class else 0))
    try:
        assert fvpatch.fv_plan_info(plan)["num_class_launches"] == 1
        for form in ("plan", "plain"):
            a = hp.to_dev(data)
            b = a.clone()
            lam = torch.empty((len(dts), T), dtype=torch.float64, device="cuda")
            for k, dt in enumerate(dts):
                if form == "plan":
                    fvpatch.fv_plan_execute(plan, a, b, dt, wl.H_DEFAULT, wl.GAMMA, lam[k])
                else:
                    fvpatch.fv_patch_batch_update(a, b, sizes, offsets, T, dim, 5, dt, wl.H_DEFAULT, wl.GAMMA, fl,
                                                  lam[k])
                a, b = b, a
            torch.cuda.synchronize()
            res[form] = (a.cpu().numpy().view(np.int64), lam.cpu().numpy().view(np.int64))
    finally:
        fvpatch.fv_plan_destroy(plan)
    assert np.array_equal(res["plan"][0], res["plain"][0])
    assert np.array_equal(res["plan"][1], res["plain"][1])
    mask = np.ones(len(data), bool)
    for t in range(T):
        mask[offsets[t]:offsets[t] + vol] = False
    assert np.array_equal(res["plan"][0][mask], data.view(np.int64)[mask])


def test_plan_replay_without_capture_is_an_error():
    from paper_2306_16731_amd import fvpatch
    b = wl.make_uniform(4, 5, seed=3)
    plan = fvpatch.fv_plan_create(b.sizes, None, 4, 2, 5)
    try:
        assert fvpatch.fv_plan_replay(plan, None, raise_on_error=False) == fvpatch.FV_ERR_INVALID_ARG
        import torch
        d = hp.to_dev(b.data)
        assert fvpatch.fv_plan_execute(plan, d, d, 1e-3, wl.H_DEFAULT, raise_on_error=False) == fvpatch.FV_ERR_OVERLAP
        assert fvpatch.fv_plan_capture_steps(plan, 2, d, d.clone(), wl.H_DEFAULT, wl.GAMMA, wl.CFL,
                                             torch.empty(4, dtype=torch.float64, device="cuda"),
                                             torch.empty(3, dtype=torch.float64, device="cuda"), None,
                                             raise_on_error=False) == fvpatch.FV_ERR_INVALID_ARG  # null stream
    finally:
        fvpatch.fv_plan_destroy(plan)


@pytest.mark.parametrize("name,mode", [("c3_2d_mixed_T200000", "per_task"), ("c4_3d_p8_T32768", "persistent")])
def test_full_size_graph_sampled(name, mode):
    """Configs 3 and 4 at their full sizes in the launch the benchmark times (the plan mode it picks,
    a captured 10-step graph with device dt): 96 sampled patches re-run by the oracle with the
    device's dt sequence, their eigenvalues, and the last dt against the device's own eigenvalues."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"full size graph: {name}, mode={mode}, 10 steps, sampled check")
    b, spec = wl.build_workload(name, seed=0)
    T, dim, steps = b.num_patches, b.dim, 10
    flags = {"persistent": 0, "per_task": fvpatch.FV_PLAN_NO_PERSIST}[mode]
    plan = fvpatch.fv_plan_create(b.sizes, b.offsets, T, dim, b.nq, flags)
    try:
        bufa = hp.to_dev(b.data)
        bufb = bufa.clone()
        lam = torch.empty(T, dtype=torch.float64, device="cuda")
        dt_dev = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        fvpatch.fv_plan_capture_steps(plan, steps, bufa, bufb, wl.H_DEFAULT, wl.GAMMA, wl.CFL, lam, dt_dev, s)
        dt_dev[0] = 1.5e-3
        torch.cuda.synchronize()
        fvpatch.fv_plan_replay(plan, s)
        s.synchronize()
        dts = dt_dev.cpu().numpy()
        lam_h = lam.cpu().numpy()
        rng = np.random.Generator(np.random.PCG64(98))
        sample = np.unique(np.concatenate([[0, T - 1], rng.choice(T, size=96, replace=False)]))
        vols = (b.sizes[sample].astype(np.int64) + 2) ** dim * b.nq
        sub_off = np.concatenate([[0], np.cumsum(vols)[:-1]]).astype(np.int64)
        sub = np.concatenate([b.data[b.offsets[t]:b.offsets[t] + v] for t, v in zip(sample, vols)])
        final = bufa if steps % 2 == 0 else bufb
        got = np.concatenate([final[int(b.offsets[t]):int(b.offsets[t]) + int(v)].cpu().numpy()
                              for t, v in zip(sample, vols)])
        assert torch.isfinite(final).all().item() and np.all(np.isfinite(lam_h))
    finally:
        fvpatch.fv_plan_destroy(plan)
    want, want_lams = oracle.run_steps(sub, b.sizes[sample], sub_off, dim, b.nq, list(dts[:steps]), wl.H_DEFAULT,
                                       wl.GAMMA, False)
    assert np.all(hp.component_errors(got, want, b.nq) <= TOL)
    assert hp.lambda_error(lam_h[sample], want_lams[-1]) <= TOL
    np.testing.assert_allclose(dts[steps], wl.CFL * wl.H_DEFAULT / (dim * float(np.max(lam_h))), rtol=TOL, atol=0)
    assert np.all(dts[1:] > 0) and np.all(np.isfinite(dts))
