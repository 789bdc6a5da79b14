"""Serving form vs the CPU oracle through the C ABI (needs a gfx950 GPU).

A server keeps a mesh's patch state on the device and applies batches (ranges
of patches, each with its own time step) in arrival order.  The final state it
reads back must equal, to 1e-12, the oracle applying the same batches in the
same order to the host copy of the mesh.
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
    print(f"[gpu-serving] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16731_amd import fvpatch
    fvpatch.load()


def oracle_replay(mesh: wl.Batch, batches, periodic=True):
    """Apply (first, count, dt) batches in order with the oracle."""
    state = mesh.data.copy()
    for first, count, dt in batches:
        idx = np.arange(first, first + count)
        sizes = mesh.sizes[idx]
        offs = mesh.offsets[idx]
        out, _ = oracle.batch_update(state, sizes, offs, mesh.dim, mesh.nq, dt, wl.H_DEFAULT, wl.GAMMA, periodic,
                                     out=state.copy(), want_lambda=False)
        for t in idx:
            n = (int(mesh.sizes[t]) + 2) ** mesh.dim * mesh.nq
            state[mesh.offsets[t]:mesh.offsets[t] + n] = out[mesh.offsets[t]:mesh.offsets[t] + n]
    return state


def batch_sequence(M, n, seed, max_count=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    seq = []
    for _ in range(n):
        first = int(rng.integers(0, M))
        count = int(rng.integers(1, (max_count or M) + 1))
        count = min(count, M - first)
        seq.append((first, count, float(rng.uniform(0.5e-3, 1.5e-3))))
    return seq


@pytest.mark.parametrize("halo", ["periodic", "from_in"])
@pytest.mark.parametrize("mode", [0, 1], ids=["fused", "plain"])
def test_server_batches_match_oracle_2d(mode, halo):
    """from_in: non-periodic with the output's halo volumes given over (whole-row writes); both
    slots of a patch start with the same halos, so the state read back is the oracle's."""
    from paper_2306_16731_amd import fvpatch as fv
    _announce(f"server 2D mixed, mode={mode}, halo={halo}")
    mesh = wl.make_mixed(300, (1, 3, 5, 9, 16, 17, 40, 63), dim=2, nq=5, seed=51)
    seq = batch_sequence(300, 40, 52)
    flags = fv.FV_HALO_PERIODIC if halo == "periodic" else fv.FV_HALO_FROM_IN
    srv = fv.fv_server_create(1 << 30, wl.GAMMA, flags, mode, 4)
    try:
        mid = fv.fv_server_add_mesh(srv, 2, 5, wl.H_DEFAULT, mesh.sizes, mesh.data)
        for first, count, dt in seq:
            fv.fv_server_submit(srv, mid, first, count, dt)
            fv.fv_server_poll(srv)
        st = fv.fv_server_drain(srv)
        assert st["completed"] == len(seq) and st["queued"] == 0 and st["inflight"] == 0
        got = fv.fv_server_read_mesh(srv, mid, np.empty_like(mesh.data))
    finally:
        fv.fv_server_destroy(srv)
    want = oracle_replay(mesh, seq, periodic=halo == "periodic")
    assert np.all(hp.component_errors(got, want, 5) <= TOL)


def test_server_batches_match_oracle_3d():
    from paper_2306_16731_amd import fvpatch as fv
    _announce("server 3D")
    mesh = wl.make_mixed(60, (2, 5, 8), dim=3, nq=5, seed=53)
    seq = batch_sequence(60, 15, 54)
    srv = fv.fv_server_create(1 << 30, wl.GAMMA, fv.FV_HALO_PERIODIC, 0, 3)
    try:
        mid = fv.fv_server_add_mesh(srv, 3, 5, wl.H_DEFAULT, mesh.sizes, mesh.data)
        for first, count, dt in seq:
            fv.fv_server_submit(srv, mid, first, count, dt)
        fv.fv_server_drain(srv)
        got = fv.fv_server_read_mesh(srv, mid, np.empty_like(mesh.data))
    finally:
        fv.fv_server_destroy(srv)
    assert np.all(hp.component_errors(got, oracle_replay(mesh, seq), 5) <= TOL)


def test_budget_admission():
    """A mesh that does not fit is refused; a tight budget queues batches (none dropped); a batch that can
    never fit is reported."""
    from paper_2306_16731_amd import fvpatch as fv
    _announce("server budget admission")
    mesh = wl.make_mixed(200, (3, 5, 9), dim=2, nq=5, seed=55)
    resident = 2 * (mesh.data.size + (mesh.data.size & 1)) * 8
    st, h = fv.fv_server_create(resident - 8, raise_on_error=False, flags=fv.FV_HALO_PERIODIC)
    assert st == fv.FV_OK
    try:
        st, mid = fv.fv_server_add_mesh(h, 2, 5, wl.H_DEFAULT, mesh.sizes, mesh.data, raise_on_error=False)
        assert st == fv.FV_ERR_BUDGET
    finally:
        fv.fv_server_destroy(h)
    # room for the mesh and about one batch of 100 patches in flight
    srv = fv.fv_server_create(resident + 100 * 44 + 8, wl.GAMMA, fv.FV_HALO_PERIODIC, 0, 8)
    try:
        mid = fv.fv_server_add_mesh(srv, 2, 5, wl.H_DEFAULT, mesh.sizes, mesh.data)
        seq = [(0, 100, 1e-3), (100, 100, 1e-3), (50, 100, 1e-3), (0, 80, 1e-3), (120, 60, 1e-3)]
        for first, count, dt in seq:
            fv.fv_server_submit(srv, mid, first, count, dt)
        st = fv.fv_server_poll(srv)
        assert st["inflight"] <= 1 and st["queued"] >= 3
        st = fv.fv_server_drain(srv)
        assert st["completed"] == len(seq) and st["peak_queued"] >= 4
        got = fv.fv_server_read_mesh(srv, mid, np.empty_like(mesh.data))
        assert np.all(hp.component_errors(got, oracle_replay(mesh, seq), 5) <= TOL)
        fv.fv_server_submit(srv, mid, 0, 200, 1e-3)  # 200 patches never fit
        st, _ = fv.fv_server_drain(srv, raise_on_error=False)
        assert st == fv.FV_ERR_BUDGET
    finally:
        fv.fv_server_destroy(srv)


@pytest.mark.parametrize("mode", [0, 1], ids=["fused", "plain"])
def test_run_trace_matches_oracle(mode):
    """A Poisson trace replayed by the C++ loop: every batch completes, latencies are recorded, and the final
    state equals the oracle applying the trace's batches in arrival order."""
    from paper_2306_16731_amd import fvpatch as fv
    from paper_2306_16731_amd import serving
    _announce(f"run_trace mode={mode}")
    mesh = wl.make_mixed(400, (3, 5, 9, 17), dim=2, nq=5, seed=56)
    trace = serving.make_trace(400.0, 0.25, [400], weights=(1,), max_batch=128, dt=(7e-4,), seed=57)
    st, log, (got,) = serving.run(mode, mesh, trace, budget=1 << 30, max_inflight=4, read_back=True)
    assert st["completed"] == len(trace) == st["submitted"] == len(log)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert np.all(log["arrival_ns"] <= log["launch_ns"]) and np.all(log["launch_ns"] <= log["done_ns"])
    seq = [(int(r["first"]), int(r["count"]), float(r["dt"])) for r in trace]
    assert np.all(hp.component_errors(got, oracle_replay(mesh, seq), 5) <= TOL)


@pytest.mark.parametrize("mode", [0, 1], ids=["fused", "plain"])
def test_mixed_2d_3d_stream_in_one_server(mode):
    """Config 5's shape at small scale: a 2D mesh of mixed sizes and a 3D 8^3 mesh registered in ONE
    server, one Poisson trace interleaving their batches 4:1; each mesh's final state equals the oracle
    applying that mesh's batches in arrival order, and the batch log covers every batch."""
    from paper_2306_16731_amd import serving
    _announce(f"mixed 2D/3D stream, one server, mode={mode}")
    m2 = wl.make_mixed(300, (3, 5, 9, 17), dim=2, nq=5, seed=58)
    m3 = wl.make_uniform(60, 8, dim=3, nq=5, seed=59)
    trace = serving.make_trace(600.0, 0.2, [300, 60], weights=(4, 1), max_batch=64, dt=(7e-4, 5e-4), seed=60)
    assert set(np.unique(trace["mesh"])) == {0, 1}
    st, log, (g2, g3) = serving.run(mode, [m2, m3], trace, budget=1 << 30, max_inflight=4, read_back=True)
    assert st["completed"] == len(trace) and st["failed"] == 0 and len(log) == len(trace)
    assert sorted(log["ticket"]) == list(range(1, len(trace) + 1))
    for mesh_id, mesh, got in ((0, m2, g2), (1, m3, g3)):
        seq = [(int(r["first"]), int(r["count"]), float(r["dt"])) for r in trace if r["mesh"] == mesh_id]
        assert np.all(hp.component_errors(got, oracle_replay(mesh, seq), 5) <= TOL), mesh_id


def _server_with_mesh(max_inflight=4, max_retries=0, deadline_ms=0.0):
    from paper_2306_16731_amd import fvpatch as fv
    mesh = wl.make_mixed(200, (3, 5, 9, 17), dim=2, nq=5, seed=61)
    srv = fv.fv_server_create(1 << 30, wl.GAMMA, fv.FV_HALO_PERIODIC, 0, max_inflight, max_retries, deadline_ms)
    mid = fv.fv_server_add_mesh(srv, 2, 5, wl.H_DEFAULT, mesh.sizes, mesh.data)
    return fv, mesh, srv, mid


def test_failed_batch_is_rerun_from_its_input_slot():
    """A batch whose completion check reports an error (forced from the host; the kernel itself runs
    normally) is re-run: drain returns, the re-run is counted, and the state equals the oracle's."""
    _announce("server failure injection: retry")
    fv, mesh, srv, mid = _server_with_mesh(max_retries=2)
    try:
        seq = [(0, 50, 1e-3), (60, 80, 9e-4), (150, 50, 1.1e-3)]
        tickets = [fv.fv_server_submit(srv, mid, *b) for b in seq]
        fv.fv_server_inject(srv, tickets[1], fv.FV_INJECT_FAIL, 2)   # fails twice, the third run succeeds
        st = fv.fv_server_drain(srv)
        assert st["completed"] == 3 and st["retried"] == 2 and st["failed"] == 0
        log = fv.fv_server_batch_log(srv)
        assert int(log[log["ticket"] == tickets[1]]["retries"][0]) == 2
        got = fv.fv_server_read_mesh(srv, mid, np.empty_like(mesh.data))
    finally:
        fv.fv_server_destroy(srv)
    assert np.all(hp.component_errors(got, oracle_replay(mesh, seq), 5) <= TOL)


def test_batch_out_of_retries_reports_launch_error_and_keeps_state():
    """With its retries spent the batch is dropped: drain returns FV_ERR_LAUNCH with the detail, the
    batch's patches keep their state from before it, and the server goes on with later batches."""
    _announce("server failure injection: retries spent")
    fv, mesh, srv, mid = _server_with_mesh(max_retries=1)
    try:
        seq = [(0, 40, 1e-3), (40, 40, 1e-3), (100, 60, 8e-4)]
        tickets = [fv.fv_server_submit(srv, mid, *b) for b in seq]
        fv.fv_server_inject(srv, tickets[1], fv.FV_INJECT_FAIL, 5)
        status, st = fv.fv_server_drain(srv, raise_on_error=False)
        assert status == fv.FV_ERR_LAUNCH and "failed" in fv.fv_last_error()
        assert st["failed"] == 1 and st["retried"] == 1
        st = fv.fv_server_drain(srv)   # the rest of the work completes
        assert st["completed"] == 2 and st["queued"] == 0 and st["inflight"] == 0
        got = fv.fv_server_read_mesh(srv, mid, np.empty_like(mesh.data))
    finally:
        fv.fv_server_destroy(srv)
    assert np.all(hp.component_errors(got, oracle_replay(mesh, [seq[0], seq[2]]), 5) <= TOL)


def test_failed_batch_whose_output_was_used_is_reported_lost():
    """A failure found after a later batch in flight has read the failed batch's output cannot be
    re-run: FV_ERR_LAUNCH names both batches, and the later batch still completes."""
    _announce("server failure injection: output already used")
    fv, mesh, srv, mid = _server_with_mesh(max_inflight=4, max_retries=3)
    try:
        t1 = fv.fv_server_submit(srv, mid, 0, 50, 1e-3)
        fv.fv_server_submit(srv, mid, 25, 50, 1e-3)   # overlaps the first batch's patches
        fv.fv_server_inject(srv, t1, fv.FV_INJECT_FAIL, 1)
        status, st = fv.fv_server_drain(srv, raise_on_error=False)
        assert status == fv.FV_ERR_LAUNCH and "lost" in fv.fv_last_error()
        assert st["failed"] == 1
        st = fv.fv_server_drain(srv)
        assert st["completed"] == 1 and st["inflight"] == 0
    finally:
        fv.fv_server_destroy(srv)


def test_deadline_ends_a_wait_for_a_batch_that_never_finishes():
    """A batch whose completion check keeps reporting "not ready" (forced from the host): poll never
    blocks; drain returns FV_ERR_LAUNCH once the deadline has passed instead of waiting forever; once
    the override is cleared the batch completes and the state equals the oracle's."""
    import time
    _announce("server deadline")
    fv, mesh, srv, mid = _server_with_mesh(max_retries=0, deadline_ms=50.0)
    try:
        seq = [(10, 100, 1e-3)]
        t = fv.fv_server_submit(srv, mid, *seq[0])
        fv.fv_server_inject(srv, t, fv.FV_INJECT_HANG)
        st = fv.fv_server_poll(srv)
        assert st["inflight"] == 1
        t0 = time.perf_counter()
        status, st = fv.fv_server_drain(srv, raise_on_error=False)
        waited = time.perf_counter() - t0
        assert status == fv.FV_ERR_LAUNCH and "deadline" in fv.fv_last_error()
        assert 0.03 <= waited < 5.0 and st["inflight"] == 1
        fv.fv_server_inject(srv, t, 0)
        st = fv.fv_server_drain(srv)
        assert st["completed"] == 1 and st["failed"] == 0
        got = fv.fv_server_read_mesh(srv, mid, np.empty_like(mesh.data))
    finally:
        fv.fv_server_destroy(srv)
    assert np.all(hp.component_errors(got, oracle_replay(mesh, seq), 5) <= TOL)


@pytest.mark.parametrize("mode", [0, 1], ids=["fused", "plain"])
def test_checkpoint_and_resume_in_a_new_server(mode):
    """Checkpoint / resume: a server replays the first half of a mixed 2D / 3D trace, its meshes are
    read back to the host and registered in a NEW server, which replays the second half.  The end state
    equals, bit for bit, one server replaying the whole trace, and the oracle to 1e-12."""
    from paper_2306_16731_amd import serving
    _announce(f"checkpoint / resume, mode={mode}")
    m2 = wl.make_mixed(240, (3, 5, 9, 17), dim=2, nq=5, seed=62)
    m3 = wl.make_uniform(40, 8, dim=3, nq=5, seed=63)
    trace = serving.make_trace(600.0, 0.2, [240, 40], weights=(4, 1), max_batch=64, dt=(7e-4, 5e-4), seed=64)
    k = len(trace) // 2
    _, _, whole = serving.run(mode, [m2, m3], trace, budget=1 << 30, max_inflight=4, read_back=True)
    _, _, (s2, s3) = serving.run(mode, [m2, m3], trace[:k], budget=1 << 30, max_inflight=4, read_back=True)
    snap2 = wl.Batch(s2, m2.sizes, m2.offsets, m2.dim, m2.nq)
    snap3 = wl.Batch(s3, m3.sizes, m3.offsets, m3.dim, m3.nq)
    rest = trace[k:].copy()
    rest["arrival_ns"] -= rest["arrival_ns"][0]
    _, log, resumed = serving.run(mode, [snap2, snap3], rest, budget=1 << 30, max_inflight=4, read_back=True)
    assert len(log) == len(rest)
    for a, b in zip(whole, resumed):
        assert np.array_equal(a, b)
    for mesh_id, mesh, got in ((0, m2, resumed[0]), (1, m3, resumed[1])):
        seq = [(int(r["first"]), int(r["count"]), float(r["dt"])) for r in trace if r["mesh"] == mesh_id]
        assert np.all(hp.component_errors(got, oracle_replay(mesh, seq), 5) <= TOL), mesh_id
