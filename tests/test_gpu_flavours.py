"""The paper's three realisations (batched, patch-wise, task graph) on the GPU through
the C ABI (needs a gfx950 GPU): bit for bit the fused kernels' results, and the
oracle's to 1e-12."""
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
    print(f"[gpu-flavours] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16731_amd import fvpatch
    fvpatch.load()


def flavour_step(flavour, data, sizes, offsets, dim, dt, h, periodic, with_lambda=True):
    import torch
    from paper_2306_16731_amd import fvpatch
    a = hp.to_dev(np.asarray(data, np.float64))
    b = a.clone()
    T = len(sizes)
    lam = torch.full((T,), -1.0, dtype=torch.float64, device="cuda") if with_lambda else None
    fvpatch.fv_flavour_update(flavour, a, b, sizes, offsets, T, dim, 5, dt, h, wl.GAMMA,
                              fvpatch.FV_HALO_PERIODIC if periodic else 0, lam)
    torch.cuda.synchronize()
    return b.cpu().numpy(), (lam.cpu().numpy() if with_lambda else None)


FLAVOURS = {"batched": 1, "patch_wise": 2, "task_graph": 3}
# An earlier realisation of the task graph as a hipGraph (assembled, instantiated, launched and
# destroyed every call) aborted the host process on the GPU machine right after
# test_task_graph_twice_in_a_row (SIGABRT from a non-Python thread, no GPU fault), and a benchmark
# sweep of it ended in a host segmentation fault; no cause was found in its code, so that form was
# removed.  The task graph is now submitted as dependent commands on streams (no graph objects).
HIPGRAPH_TASK_GRAPH_OFF = ("tests the removed hipGraph task-graph form, which aborted the host process on "
                           "the GPU box with no cause shown in its code")
CASES = [(2, 4), (2, 6), (2, 8), (2, 16), (3, 4), (3, 6), (3, 8)]


@pytest.mark.parametrize("name", list(FLAVOURS))
@pytest.mark.parametrize("dim,p", CASES)
@pytest.mark.parametrize("periodic", [False, True])
def test_flavour_matches_fused_and_oracle(name, dim, p, periodic):
    _announce(f"{name} dim={dim} p={p} periodic={periodic}")
    T = 37 if name != "task_graph" else 11
    b = wl.make_uniform(T, p, dim=dim, nq=5, seed=50 + p + dim)
    dt, h = 1.1e-3, wl.H_DEFAULT
    got, lam = flavour_step(FLAVOURS[name], b.data, b.sizes, None, dim, dt, h, periodic)
    fused, flam = hp.gpu_step(b.data, b.sizes, b.offsets, dim, 5, dt, h, wl.GAMMA, periodic)
    assert np.array_equal(got, fused), "not bitwise equal to the fused kernel"
    assert np.array_equal(lam, flam)
    want, wlam = oracle.batch_update(b.data, b.sizes, b.offsets, dim, 5, dt, h, wl.GAMMA, periodic)
    assert np.all(hp.component_errors(got, want, 5) <= TOL)
    assert hp.lambda_error(lam, wlam) <= TOL


@pytest.mark.parametrize("name", list(FLAVOURS))
def test_flavour_gapped_offsets_and_no_reduction(name):
    """Patches at gapped (odd) offsets: bytes between them untouched; without lambda."""
    _announce(f"{name} gapped offsets")
    p, dim, T = 6, 2, 23
    rng = np.random.Generator(np.random.PCG64(60))
    compact = wl.make_uniform(T, p, dim=dim, nq=5, seed=61)
    vol = (p + 2) ** dim * 5
    starts = np.cumsum(np.concatenate([[3], vol + rng.integers(0, 5, size=T - 1)])).astype(np.int64)
    data = rng.uniform(-1, 1, int(starts[-1] + vol + 4))
    for t in range(T):
        data[starts[t]:starts[t] + vol] = compact.data[t * vol:(t + 1) * vol]
    got, _ = flavour_step(FLAVOURS[name], data, compact.sizes, starts, dim, 1e-3, wl.H_DEFAULT, True,
                          with_lambda=False)
    mask = np.ones(len(data), bool)
    for t in range(T):
        mask[starts[t]:starts[t] + vol] = False
    assert np.array_equal(got[mask], data[mask])
    want, _ = oracle.batch_update(data, compact.sizes, starts, dim, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, True)
    assert np.all(hp.component_errors(got[~mask], want[~mask], 5) <= TOL)


@pytest.mark.skip(reason=HIPGRAPH_TASK_GRAPH_OFF)
def test_task_graph_twice_in_a_row():
    """The second call waits for the first call's graph before replacing it."""
    from paper_2306_16731_amd import fvpatch
    b = wl.make_uniform(9, 4, dim=3, nq=5, seed=62)
    g1, l1 = flavour_step(3, b.data, b.sizes, None, 3, 1e-3, wl.H_DEFAULT, False)
    g2, l2 = flavour_step(3, g1, b.sizes, None, 3, 1e-3, wl.H_DEFAULT, False)
    s1, _ = oracle.batch_update(b.data, b.sizes, b.offsets, 3, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, False)
    s2, wl2 = oracle.batch_update(s1, b.sizes, b.offsets, 3, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, False)
    assert np.all(hp.component_errors(g2, s2, 5) <= TOL)
    assert hp.lambda_error(l2, wl2) <= TOL


def test_task_submission_calls_in_a_row_buffers_freed():
    """The dependent-command task graph: three calls queued on one stream with no synchronisation
    between them (the second reads the first's output), then the first call's buffers freed and a
    larger batch (the flux workspace grows): every result equals the oracle's chain."""
    import torch
    from paper_2306_16731_amd import fvpatch
    _announce("task graph: calls in a row")
    b = wl.make_uniform(9, 4, dim=3, nq=5, seed=62)
    a = hp.to_dev(b.data)
    c = a.clone()
    d = a.clone()
    lam = torch.full((9,), -1.0, dtype=torch.float64, device="cuda")
    for src, dst in ((a, c), (c, d), (d, a)):
        fvpatch.fv_flavour_update(3, src, dst, b.sizes, None, 9, 3, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, 0, lam)
    torch.cuda.synchronize()
    got = a.cpu().numpy()
    s_ = b.data
    for _ in range(3):
        s_, wl_ = oracle.batch_update(s_, b.sizes, b.offsets, 3, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, False)
    assert np.all(hp.component_errors(got, s_, 5) <= TOL)
    assert hp.lambda_error(lam.cpu().numpy(), wl_) <= TOL
    del a, c, d
    torch.cuda.empty_cache()
    b2 = wl.make_uniform(300, 6, dim=3, nq=5, seed=63)
    g2, l2 = flavour_step(3, b2.data, b2.sizes, None, 3, 1e-3, wl.H_DEFAULT, True)
    w2, wl2 = oracle.batch_update(b2.data, b2.sizes, b2.offsets, 3, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, True)
    assert np.all(hp.component_errors(g2, w2, 5) <= TOL)
    assert hp.lambda_error(l2, wl2) <= TOL
