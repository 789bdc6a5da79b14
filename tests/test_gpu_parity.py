"""HIP path vs the CPU oracle, element by element, through the C ABI (needs a gfx950 GPU).

Tolerance: every unknown's max-norm error, relative to that unknown's max-norm
over the batch, must be <= 1e-12, and so must the per-patch eigenvalues'.
Both sides get the same seeded inputs and the same time-step sequence.  The
expected error is ~1e-15 (the kernel fuses multiply-adds and uses 1/rho times
m instead of m / rho; the oracle rounds every operation separately).
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2306_16731_amd import workloads as wl
from tests import hip_path as hp
from tests import invariants as inv

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _announce(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


def dt_sequence(batch, steps, periodic, h=wl.H_DEFAULT):
    """dt_{n+1} = CFL h / (d max lambda_n) along the oracle's own trajectory."""
    lam0 = oracle.batch_lambda(batch.data, batch.sizes, batch.offsets, batch.dim, batch.nq)
    dts = [wl.CFL * h / (batch.dim * float(np.max(lam0)))]
    state = batch.data.copy()
    buf = state.copy()
    for _ in range(steps - 1):
        buf, lam = oracle.batch_update(state, batch.sizes, batch.offsets, batch.dim, batch.nq, dts[-1], h,
                                       wl.GAMMA, periodic, out=buf)
        state, buf = buf, state
        dts.append(wl.CFL * h / (batch.dim * float(np.max(lam))))
    return dts


def compare_run(batch, steps, periodic, pass_offsets=True):
    dts = dt_sequence(batch, steps, periodic)
    want, want_lams = oracle.run_steps(batch.data, batch.sizes, batch.offsets, batch.dim, batch.nq, dts,
                                       wl.H_DEFAULT, wl.GAMMA, periodic)
    got, got_lams = hp.gpu_run_steps(batch.data, batch.sizes, batch.offsets, batch.dim, batch.nq, dts,
                                     wl.H_DEFAULT, wl.GAMMA, periodic, pass_offsets=pass_offsets)
    errs = hp.component_errors(got, want, batch.nq)
    lerr = max(hp.lambda_error(g, w) for g, w in zip(got_lams, want_lams))
    assert np.all(errs <= TOL), errs
    assert lerr <= TOL, lerr
    return errs, lerr


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16731_amd import fvpatch
    fvpatch.load()


def test_c1_golden_and_oracle():
    _announce("c1: 16 x 3^2, 2D, one step")
    from tests.golden import make_golden as mg
    b, dt, want, want_lam = mg.c1_case(0)
    for pass_offsets in (True, False):
        got, lam = hp.gpu_step(b.data, b.sizes, b.offsets, 2, 5, dt, wl.H_DEFAULT, wl.GAMMA, False,
                               pass_offsets=pass_offsets)
        assert np.all(hp.component_errors(got, want, 5) <= TOL)
        assert hp.lambda_error(lam, want_lam) <= TOL


@pytest.mark.parametrize("pass_offsets", [False, True])
def test_c2_reduced_periodic_10_steps(pass_offsets):
    _announce(f"c2 reduced: 300 x 16^2, 10 steps, periodic, offsets={pass_offsets}")
    b, _ = wl.build_workload("c2_2d_p16_T65536", seed=1, num_patches=300)
    compare_run(b, 10, True, pass_offsets)


def test_c3_reduced_mixed_sizes():
    _announce("c3 reduced: 1500 mixed {3,5,9,17}^2, 10 steps")
    b, _ = wl.build_workload("c3_2d_mixed_T200000", seed=2, num_patches=1500)
    compare_run(b, 10, False)


@pytest.mark.parametrize("periodic", [False, True])
def test_c4_reduced_3d(periodic):
    _announce(f"c4 reduced: 200 x 8^3, 10 steps, periodic={periodic}")
    b, _ = wl.build_workload("c4_3d_p8_T32768", seed=3, num_patches=200)
    compare_run(b, 10, periodic, pass_offsets=False)


def test_two_d_n4():
    _announce("2D N=4: 257 x 7^2, 5 steps")
    b = wl.make_uniform(257, 7, dim=2, nq=4, seed=4, pulse=True)
    compare_run(b, 5, True)


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 31), (2, 62), (2, 63), (2, 64), (3, 1), (3, 2), (3, 7),
                                   (3, 14), (3, 15), (3, 24)])
def test_sizes_edge(dim, p):
    _announce(f"edge sizes: dim={dim} p={p}")
    T = 5 if p > 20 else 37
    b = wl.make_uniform(T, p, dim=dim, nq=5, seed=10 + p)
    compare_run(b, 2, True, pass_offsets=False)
    compare_run(b, 1, False, pass_offsets=True)


def test_ragged_offsets_with_gaps_unsorted_and_odd():
    """Patches at unsorted offsets with gaps, some starting at odd doubles (8- not 16-byte aligned)."""
    _announce("ragged offsets")
    rng = np.random.Generator(np.random.PCG64(77))
    sizes = rng.choice(np.array([1, 3, 4, 9, 16, 17, 30], np.int32), size=211)
    vols = (sizes.astype(np.int64) + 2) ** 2 * 5
    gaps = rng.integers(0, 7, size=len(sizes))
    starts = np.cumsum(np.concatenate([[3], (vols + gaps)[:-1]])).astype(np.int64)
    perm = rng.permutation(len(sizes))
    total = int(starts[-1] + vols[-1] + 5)
    compact = wl.make_batch(sizes, 2, 5, seed=78)
    data = rng.uniform(-1, 1, total)  # filler between patches: must stay untouched
    for t in range(len(sizes)):
        data[starts[t]:starts[t] + vols[t]] = compact.data[compact.offsets[t]:compact.offsets[t] + vols[t]]
    s2, o2 = sizes[perm], starts[perm]
    dts = [1.1e-3, 1.3e-3, 0.9e-3]
    want, want_lams = oracle.run_steps(data, s2, o2, 2, 5, dts, wl.H_DEFAULT, wl.GAMMA, True)
    got, got_lams = hp.gpu_run_steps(data, s2, o2, 2, 5, dts, wl.H_DEFAULT, wl.GAMMA, True)
    mask = np.ones(total, bool)
    for t in range(len(sizes)):
        mask[starts[t]:starts[t] + vols[t]] = False
    assert np.array_equal(got[mask], data[mask]), "bytes outside the patches were written"
    inside = ~mask
    assert np.all(hp.component_errors(got[inside], want[inside], 5) <= TOL)
    assert max(hp.lambda_error(g, w) for g, w in zip(got_lams, want_lams)) <= TOL


@pytest.mark.parametrize("dim,p,base,gap", [(2, 16, 0, 0), (2, 16, 1, 6), (2, 17, 2, 3), (2, 9, 3, 1), (3, 8, 1, 10)])
@pytest.mark.parametrize("periodic", [False, True])
def test_evenly_spaced_offsets(dim, p, base, gap, periodic):
    """Equal sizes at evenly spaced offsets (patch t at base + t (patch + gap)) run as a contiguous
    launch from the first patch, with no descriptors uploaded: the result must equal, bit for bit,
    the same patches at offsets that are not evenly spaced (the descriptor path), leave the gaps
    untouched, and match the oracle."""
    _announce(f"evenly spaced offsets dim={dim} p={p} base={base} gap={gap} periodic={periodic}")
    T = 97
    vol = (p + 2) ** dim * 5
    compact = wl.make_uniform(T, p, dim=dim, seed=61)
    rng = np.random.Generator(np.random.PCG64(62))
    layouts = {"even": base + np.arange(T, dtype=np.int64) * (vol + gap)}
    jitter = np.concatenate([[0], rng.integers(0, 3, size=T - 1)])   # one uneven gap at least
    jitter[T // 2] = 1
    layouts["uneven"] = base + np.arange(T, dtype=np.int64) * (vol + gap) + np.cumsum(jitter)
    results = {}
    for name, offs in layouts.items():
        total = int(offs[-1] + vol + 4)
        data = rng.uniform(-1, 1, total)
        for t in range(T):
            data[offs[t]:offs[t] + vol] = compact.data[t * vol:(t + 1) * vol]
        got, lam = hp.gpu_step(data, compact.sizes, offs, dim, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, periodic)
        mask = np.ones(total, bool)
        for t in range(T):
            mask[offs[t]:offs[t] + vol] = False
        assert np.array_equal(got[mask], data[mask]), (name, "bytes outside the patches were written")
        results[name] = (np.concatenate([got[o:o + vol] for o in offs]), lam)
    assert np.array_equal(results["even"][0], results["uneven"][0])
    assert np.array_equal(results["even"][1], results["uneven"][1])
    want, want_lam = oracle.batch_update(compact.data, compact.sizes, compact.offsets, dim, 5, 1.2e-3,
                                         wl.H_DEFAULT, wl.GAMMA, periodic)
    assert np.all(hp.component_errors(results["even"][0], want, 5) <= TOL)
    assert hp.lambda_error(results["even"][1], want_lam) <= TOL


@pytest.mark.parametrize("kernel", ["tile", "wave", "block"])
@pytest.mark.parametrize("p,gap", [(7, 1), (17, 3), (9, 1)])
def test_evenly_spaced_offsets_tuned_odd_patches(kernel, p, gap):
    """Patches with an odd number of doubles at an even spacing (the gap makes the stride even)
    under every runtime-size kernel the tuner may install: the evenly spaced fast path must not
    take 16-byte accesses for them; the result equals the descriptor path's and the oracle's."""
    from paper_2306_16731_amd import fvpatch
    _announce(f"evenly spaced odd patches p={p} gap={gap} kernel={kernel}")
    kid = {"tile": fvpatch.FV_KERNEL_TILE, "wave": fvpatch.FV_KERNEL_WAVE, "block": fvpatch.FV_KERNEL_BLOCK}[kernel]
    T, dim = 67, 2
    vol = (p + 2) ** dim * 5
    assert vol % 2 == 1 and (vol + gap) % 2 == 0
    compact = wl.make_uniform(T, p, dim=dim, seed=63)
    offs = np.arange(T, dtype=np.int64) * (vol + gap)
    total = int(offs[-1] + vol + 2)
    data = np.random.Generator(np.random.PCG64(64)).uniform(-1, 1, total)
    for t in range(T):
        data[offs[t]:offs[t] + vol] = compact.data[t * vol:(t + 1) * vol]
    fvpatch.fv_set_tuning(dim, 5, p, {"kernel": kid})
    try:
        got, lam = hp.gpu_step(data, compact.sizes, offs, dim, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, False)
    finally:
        fvpatch.fv_set_tuning(dim, 5, p, None)
    mask = np.ones(total, bool)
    for t in range(T):
        mask[offs[t]:offs[t] + vol] = False
    assert np.array_equal(got[mask], data[mask]), "bytes outside the patches were written"
    want, want_lam = oracle.batch_update(compact.data, compact.sizes, compact.offsets, dim, 5, 1.2e-3,
                                         wl.H_DEFAULT, wl.GAMMA, False)
    got_c = np.concatenate([got[o:o + vol] for o in offs])
    inner = np.zeros((p + 2, p + 2), bool)
    inner[1:-1, 1:-1] = True
    sel = np.tile(np.repeat(inner.ravel(), 5), T)
    assert np.all(hp.component_errors(got_c[sel], want[sel], 5) <= TOL)
    assert hp.lambda_error(lam, want_lam) <= TOL


def test_single_patch_and_zero_patches():
    import torch
    from paper_2306_16731_amd import fvpatch
    b = wl.make_uniform(1, 16, seed=5)
    compare_run(b, 3, True, pass_offsets=False)
    d = torch.zeros(10, dtype=torch.float64, device="cuda")
    assert fvpatch.fv_patch_batch_update(d, d, [], None, 0, 2, 5, 1e-3, 1 / 48) == 0


def test_deterministic_bitwise():
    b = wl.make_mixed(700, seed=6)
    r1 = hp.gpu_step(b.data, b.sizes, b.offsets, 2, 5, 1.3e-3, wl.H_DEFAULT, wl.GAMMA, True)
    r2 = hp.gpu_step(b.data, b.sizes, b.offsets, 2, 5, 1.3e-3, wl.H_DEFAULT, wl.GAMMA, True)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])


def test_c2_full_size_sampled():
    """Config 2 at its full size (65536 x 16^2, 10 steps, periodic) in the launch the benchmark
    times; 96 sampled patches re-run by the oracle with the same dt sequence."""
    _announce("c2 full size: 65536 x 16^2, 10 steps, sampled check")
    import torch
    from paper_2306_16731_amd import fvpatch
    b, spec = wl.build_workload("c2_2d_p16_T65536", seed=0)
    T = b.num_patches
    rng = np.random.Generator(np.random.PCG64(99))
    sample = np.sort(rng.choice(T, size=96, replace=False))
    sample = np.unique(np.concatenate([[0, T - 1], sample]))
    stride = int(b.offsets[1])
    sub = np.concatenate([b.data[t * stride:(t + 1) * stride] for t in sample])
    sub_sizes = b.sizes[sample]
    sub_off = np.arange(len(sample), dtype=np.int64) * stride
    dts = [1.9e-3 * (1 + 0.01 * s) for s in range(10)]
    want, want_lams = oracle.run_steps(sub, sub_sizes, sub_off, 2, 5, dts, wl.H_DEFAULT, wl.GAMMA, True)
    a = hp.to_dev(b.data)
    bb = a.clone()
    lam = torch.empty(T, dtype=torch.float64, device="cuda")
    for dt in dts:
        fvpatch.fv_patch_batch_update(a, bb, b.sizes, None, T, 2, 5, dt, wl.H_DEFAULT, wl.GAMMA,
                                      fvpatch.FV_HALO_PERIODIC, lam)
        a, bb = bb, a
    torch.cuda.synchronize()
    idx = torch.from_numpy(sample).to("cuda")
    got = a.view(T, stride)[idx].cpu().numpy().reshape(-1)
    got_lam = lam[idx].cpu().numpy()
    assert np.all(hp.component_errors(got, want, 5) <= TOL)
    assert hp.lambda_error(got_lam, want_lams[-1]) <= TOL
    # every patch's state stays physical and finite
    assert torch.isfinite(a).all().item() and torch.isfinite(lam).all().item()
    del a, bb


# --------------------------------------------------------------------- the invariant suite on the HIP path
INV_CASES = [(2, 5), (2, 4), (3, 5)]


@pytest.mark.parametrize("step", [hp.gpu_step, hp.gpu_step_contiguous], ids=["offsets", "contiguous"])
@pytest.mark.parametrize("dim,nq", INV_CASES)
def test_invariants_on_gpu(step, dim, nq):
    _announce(f"invariants dim={dim} nq={nq} step={step.__name__}")
    inv.check_constant_state(step, dim, nq)
    inv.check_conservation(step, dim, nq)
    inv.check_mirror(step, dim, nq)
    inv.check_permutation(step, dim, nq)
    inv.check_corner_independence(step, dim, nq)
    inv.check_lambda_reduction(step, dim, nq)
    inv.check_nan_propagates(step, dim, nq)


@pytest.mark.parametrize("dim,p", [(2, 16), (2, 9), (2, 3), (3, 8), (3, 4)])
def test_invariants_on_gpu_fixed_sizes(dim, p):
    """The invariants at sizes the fixed-size kernels serve by default."""
    _announce(f"invariants at fixed size dim={dim} p={p}")
    inv.check_constant_state(hp.gpu_step, dim, 5, p=p)
    inv.check_conservation(hp.gpu_step, dim, 5, p=p)
    inv.check_mirror(hp.gpu_step, dim, 5, p=p)
    inv.check_permutation(hp.gpu_step, dim, 5, p=p)
    inv.check_corner_independence(hp.gpu_step, dim, 5, p=p)
    inv.check_lambda_reduction(hp.gpu_step, dim, 5, p=p)
    inv.check_nan_propagates(hp.gpu_step, dim, 5, p=p)


def test_dimension_reduction_and_closed_form_on_gpu():
    inv.check_dimension_reduction(hp.gpu_step)
    inv.check_passive_scalar(hp.gpu_step)
    inv.check_passive_scalar(hp.gpu_step, u0=0.44, p0=1.21, seed=11)


def test_acoustic_convergence_on_gpu():
    inv.check_acoustic_convergence(hp.gpu_step, 2, 5, (1, 1), sizes=(16, 32, 64))
    # 3D: patches above 24^3 are out of range, so compare the error itself with the oracle's
    for p in (8, 16, 24):
        e_gpu = inv.acoustic_error(hp.gpu_step, p, 3, 5, (0, 0, 1))
        e_ora = inv.acoustic_error(lambda *a: oracle.batch_update(*a), p, 3, 5, (0, 0, 1))
        assert abs(e_gpu - e_ora) <= 1e-9 * e_ora, (p, e_gpu, e_ora)


# --------------------------------------------------------------------- every kernel variant the tuner may pick
VARIANTS = [
    (2, 16, dict(kernel=3, block=256)), (2, 16, dict(kernel=3, block=512)), (2, 16, dict(kernel=2, block=256, prefetch=1)),
    (2, 16, dict(kernel=2, block=64, prefetch=4)), (2, 16, dict(kernel=1, block=128)), (2, 16, dict(kernel=1, block=320)),
    (2, 16, dict(kernel=2, block=256, prefetch=4, rows=1)), (2, 16, dict(kernel=2, block=128, prefetch=2, rows=16)),
    (2, 17, dict(kernel=2, block=256, prefetch=3, rows=5)), (2, 3, dict(kernel=2, block=64, prefetch=1, rows=3)),
    (2, 62, dict(kernel=2, block=64, prefetch=2, rows=7)),
    (2, 3, dict(kernel=3, block=64)), (2, 3, dict(kernel=3, block=256)), (2, 5, dict(kernel=3, block=128)),
    (2, 9, dict(kernel=3, block=128)), (2, 17, dict(kernel=3, block=320)), (2, 17, dict(kernel=3, block=640)),
    (2, 32, dict(kernel=3, block=1024)), (2, 30, dict(kernel=2, block=128, prefetch=2)), (2, 17, dict(kernel=1, block=64)),
    (3, 8, dict(kernel=1, block=128)), (3, 8, dict(kernel=1, block=512)),
    (2, 3, dict(kernel=4)), (2, 5, dict(kernel=4)), (2, 9, dict(kernel=4)), (2, 16, dict(kernel=4)),
    (2, 17, dict(kernel=4)), (3, 4, dict(kernel=4)), (3, 6, dict(kernel=4)), (3, 8, dict(kernel=4)),
    (3, 4, dict(kernel=1, block=128)), (3, 6, dict(kernel=1, block=128)),
]


@pytest.mark.parametrize("dim,p,tuning", VARIANTS, ids=[f"{d}d-p{p}-{t}" for d, p, t in VARIANTS])
def test_kernel_variants(dim, p, tuning):
    from paper_2306_16731_amd import fvpatch
    _announce(f"variant dim={dim} p={p} {tuning}")
    try:
        fvpatch.fv_set_tuning(dim, 5, p, tuning)
        b = wl.make_uniform(23, p, dim=dim, nq=5, seed=40 + p)
        compare_run(b, 2, True, pass_offsets=False)
        compare_run(b, 1, False, pass_offsets=True)
        inv.check_constant_state(hp.gpu_step, dim, 5, p=p, T=3)
    finally:
        fvpatch.fv_set_tuning(dim, 5, p, None)


# --------------------------------------------------------------------- fixed-size build vs runtime-size kernel
@pytest.mark.parametrize("p", [3, 5, 9, 16, 17])
@pytest.mark.parametrize("periodic", [False, True])
def test_fixed_size_kernel_matches_runtime_size_kernel_bitwise(p, periodic):
    """Both forms of the wave kernel round identically, so their results agree bit for bit: a ragged
    last wave (spare slots), patches at gapped offsets (odd and even starts) and contiguous ones."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"fixed vs runtime size: p={p} periodic={periodic}")
    ppw = 64 // (p + 2)
    T = 4 * 4 * ppw + ppw // 2 + 1
    rng = np.random.Generator(np.random.PCG64(90 + p))
    compact = wl.make_uniform(T, p, dim=2, nq=5, seed=91 + p)
    vol = (p + 2) ** 2 * 5
    starts = np.cumsum(np.concatenate([[1], vol + rng.integers(0, 4, size=T - 1)])).astype(np.int64)
    data = rng.uniform(-1, 1, int(starts[-1] + vol + 3))
    for t in range(T):
        data[starts[t]:starts[t] + vol] = compact.data[t * vol:(t + 1) * vol]
    sizes = np.full(T, p, np.int32)
    results = {}
    try:
        for kernel in (fvpatch.FV_KERNEL_FIXED, fvpatch.FV_KERNEL_WAVE):
            fvpatch.fv_set_tuning(2, 5, p, dict(kernel=kernel, block=0, prefetch=0, rows=0))
            results[kernel] = (hp.gpu_step(data, sizes, starts, 2, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, periodic),
                               hp.gpu_step(compact.data, sizes, None, 2, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, periodic,
                                           pass_offsets=False))
    finally:
        fvpatch.fv_set_tuning(2, 5, p, None)
    (fo, fc), (wo, wc) = results[fvpatch.FV_KERNEL_FIXED], results[fvpatch.FV_KERNEL_WAVE]
    for f, w in ((fo, wo), (fc, wc)):
        assert np.array_equal(f[0], w[0]) and np.array_equal(f[1], w[1])
    mask = np.ones(len(data), bool)
    for t in range(T):
        mask[starts[t]:starts[t] + vol] = False
    assert np.array_equal(fo[0][mask], data[mask]), "bytes outside the patches were written"
    want, want_lam = oracle.batch_update(compact.data, sizes, compact.offsets, 2, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA,
                                         periodic)
    assert np.all(hp.component_errors(fc[0], want, 5) <= TOL)
    assert hp.lambda_error(fc[1], want_lam) <= TOL


@pytest.mark.parametrize("p", [4, 6, 8])
@pytest.mark.parametrize("periodic", [False, True])
def test_fixed_3d_kernel_matches_block_kernel_bitwise(p, periodic):
    """The 3D one-wave-per-cross-section kernel and the plane-marching block kernel round
    identically: bit-equal results, with a ragged last wave, gapped offsets and contiguous ones."""
    from paper_2306_16731_amd import fvpatch
    _announce(f"3D fixed vs block: p={p} periodic={periodic}")
    lanes = (p + 2) ** 2 // 2
    ppw = 64 // lanes
    T = 7 * ppw + max(ppw - 1, 1)
    rng = np.random.Generator(np.random.PCG64(190 + p))
    compact = wl.make_uniform(T, p, dim=3, nq=5, seed=191 + p)
    vol = (p + 2) ** 3 * 5
    starts = np.cumsum(np.concatenate([[1], vol + rng.integers(0, 4, size=T - 1)])).astype(np.int64)
    data = rng.uniform(-1, 1, int(starts[-1] + vol + 3))
    for t in range(T):
        data[starts[t]:starts[t] + vol] = compact.data[t * vol:(t + 1) * vol]
    sizes = np.full(T, p, np.int32)
    results = {}
    try:
        for kernel in (fvpatch.FV_KERNEL_FIXED, fvpatch.FV_KERNEL_BLOCK):
            fvpatch.fv_set_tuning(3, 5, p, dict(kernel=kernel, block=0, prefetch=0, rows=0))
            results[kernel] = (hp.gpu_step(data, sizes, starts, 3, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, periodic),
                               hp.gpu_step(compact.data, sizes, None, 3, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, periodic,
                                           pass_offsets=False))
    finally:
        fvpatch.fv_set_tuning(3, 5, p, None)
    (fo, fc), (bo, bc) = results[fvpatch.FV_KERNEL_FIXED], results[fvpatch.FV_KERNEL_BLOCK]
    for f, b in ((fo, bo), (fc, bc)):
        assert np.array_equal(f[1], b[1])
        assert np.array_equal(f[0], b[0])
    mask = np.ones(len(data), bool)
    for t in range(T):
        mask[starts[t]:starts[t] + vol] = False
    assert np.array_equal(fo[0][mask], data[mask]), "bytes outside the patches were written"
    want, want_lam = oracle.batch_update(compact.data, sizes, compact.offsets, 3, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA,
                                         periodic)
    assert np.all(hp.component_errors(fc[0], want, 5) <= TOL)
    assert hp.lambda_error(fc[1], want_lam) <= TOL


def _patch_masks(total, sizes, offsets, dim, nq):
    """Boolean masks over the buffer: interior volumes, x-halo volumes of interior rows (2D), and
    every volume of the patches."""
    interior = np.zeros(total, bool)
    xhalo = np.zeros(total, bool)
    inside = np.zeros(total, bool)
    for p, o in zip(sizes, offsets):
        W = int(p) + 2
        blk = np.zeros((W,) * dim + (nq,), bool)
        inner = blk.copy()
        inner[(slice(1, -1),) * dim] = True
        xh = blk.copy()
        if dim == 2:
            xh[1:-1, 0] = True
            xh[1:-1, -1] = True
        else:   # axes (k, j, i): the x-halo volumes of the interior rows of the interior layers
            xh[1:-1, 1:-1, 0] = True
            xh[1:-1, 1:-1, -1] = True
        n = W ** dim * nq
        interior[o:o + n] = inner.reshape(-1)
        xhalo[o:o + n] = xh.reshape(-1)
        inside[o:o + n] = True
    return interior, xhalo, inside


@pytest.mark.parametrize("case", ["plain-3", "plain-5", "plain-9", "plain-16", "plain-17", "plain-7", "plain-30",
                                  "plain-3d-8", "plain-3d-4", "plain-3d-6", "plan-mixed"])
def test_halo_from_in(case):
    """FV_HALO_FROM_IN: the interior and lambda equal, bit for bit, a step without the flag; every
    output halo volume is either untouched or equal to the input's (the 2D row-marching kernels,
    fixed-size and runtime-size, and the 3D interior-mapped kernel (p = 4, 8) write the x-halo volumes
    of the interior rows; the other kernels none); bytes between patches stay untouched."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce(f"halo from input: {case}")
    rng = np.random.Generator(np.random.PCG64(71))
    dim = 3 if case.startswith("plain-3d") else 2
    if case == "plan-mixed":
        sizes = rng.choice(np.array([3, 5, 7, 9, 16, 17], np.int32), size=600)
    else:
        sizes = np.full(150, int(case.split("-")[-1]), np.int32)
    vols = (sizes.astype(np.int64) + 2) ** dim * 5
    offs = np.cumsum(np.concatenate([[2], (vols + 4)[:-1]])).astype(np.int64)
    total = int(offs[-1] + vols[-1] + 3)
    compact = wl.make_batch(sizes, dim, 5, seed=72)
    data = rng.uniform(-1, 1, total)
    for t in range(len(sizes)):
        data[offs[t]:offs[t] + vols[t]] = compact.data[compact.offsets[t]:compact.offsets[t] + vols[t]]
    filler = rng.uniform(-1, 1, total)   # the output buffer's prior contents
    res = {}
    for flag in (0, fvpatch.FV_HALO_FROM_IN):
        a = hp.to_dev(data)
        b = hp.to_dev(filler)
        lam = torch.empty(len(sizes), dtype=torch.float64, device="cuda")
        if case == "plan-mixed":
            plan = fvpatch.fv_plan_create(sizes, offs, len(sizes), dim, 5, flag | fvpatch.FV_PLAN_NO_PERSIST)
            try:
                fvpatch.fv_plan_execute(plan, a, b, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, lam)
                torch.cuda.synchronize()
            finally:
                fvpatch.fv_plan_destroy(plan)
        else:
            fvpatch.fv_patch_batch_update(a, b, sizes, offs, len(sizes), dim, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA,
                                          flag, lam)
            torch.cuda.synchronize()
        res[flag] = (b.cpu().numpy(), lam.cpu().numpy())
    interior, xhalo, inside = _patch_masks(total, sizes, offs, dim, 5)
    (o0, l0), (o1, l1) = res[0], res[fvpatch.FV_HALO_FROM_IN]
    assert np.array_equal(o1[interior], o0[interior]) and np.array_equal(l1, l0)
    halo = inside & ~interior
    assert np.array_equal(o0[halo], filler[halo])                       # without the flag: untouched
    assert np.all((o1[halo] == filler[halo]) | (o1[halo] == data[halo]))
    assert np.array_equal(o1[~inside], filler[~inside])                 # between patches: untouched
    whole = (sizes + 2 <= 64) if dim == 2 else np.isin(sizes, [4, 8])
    if whole.any():   # the whole-row form ran: the x-halo volumes of those patches took the input's values
        xm = np.zeros(total, bool)
        for t in np.nonzero(whole)[0]:
            xm[offs[t]:offs[t] + vols[t]] = xhalo[offs[t]:offs[t] + vols[t]]
        assert np.array_equal(o1[xm], data[xm])
    want, want_lam = oracle.batch_update(data, sizes, offs, dim, 5, 1.2e-3, wl.H_DEFAULT, wl.GAMMA, False)
    assert np.all(hp.component_errors(o1[interior], want[interior], 5) <= TOL)
    assert hp.lambda_error(l1, want_lam) <= TOL
