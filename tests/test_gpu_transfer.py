"""Patches in host memory through fv_host_patches_update (needs a gfx950 GPU).

Both transfer modes against the CPU oracle (1e-12 relative, as elsewhere) and,
bit for bit, against fv_patch_batch_update on the same patches already in
device memory: moving patches is a copy and may change nothing.  Chunk sizes
are chosen so that a batch spans several chunks with a short last one, with
fewer slots than chunks (slots are reused) and one slot (no overlap)."""
from __future__ import annotations

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
    print(f"[gpu-transfer] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16731_amd import fvpatch
    fvpatch.load()


def run_host(batch, mode, chunk_patches=0, slots=0, threads=0, periodic=False, dt=1.1e-3, seed=0,
             want_lambda=True):
    from paper_2306_16731_amd import fvpatch
    src = wl.scatter_to_host(batch, seed=seed)
    dst = [np.full_like(a, np.nan) for a in src]
    T = batch.num_patches
    lam = np.full(T, -1.0) if want_lambda else None
    pbytes = src[0].nbytes if T else 8
    # a chunk of chunk_patches and a half patches: whole patches only, the half is left over
    cfg = {"mode": mode, "slots": slots, "host_threads": threads,
           "chunk_bytes": int(pbytes * chunk_patches + pbytes // 2) if chunk_patches else 0}
    stats = {}
    fvpatch.fv_host_patches_update(src, dst, batch.sizes, T, batch.dim, batch.nq, dt, wl.H_DEFAULT, wl.GAMMA,
                                   fvpatch.FV_HALO_PERIODIC if periodic else 0, lam, config=cfg, stats=stats)
    return src, dst, lam, stats


def gathered(batch, arrays):
    return np.concatenate(arrays) if arrays else np.zeros(0)


CASES = [  # (p, dim, T, mode, chunk patches, slots per thread, threads)
    (16, 2, 37, "pipelined", 5, 3, 4),     # fixed-size kernel, 8 chunks over 4 threads, last one short
    (7, 2, 23, "pipelined", 4, 2, 1),      # runtime-size kernel, one thread: slots reused in turn
    (3, 2, 50, "pipelined", 7, 1, 8),      # one slot per thread: no overlap within a thread
    (16, 2, 29, "pipelined", 0, 0, 0),     # defaults: one chunk
    (16, 2, 64, "pipelined", 1, 2, 16),    # one patch per chunk, more threads than the default pool
    (8, 3, 19, "pipelined", 3, 4, 3),      # 3D fixed-size kernel
    (5, 3, 11, "pipelined", 2, 8, 2),      # 3D runtime size, more slots than chunks need
    (16, 2, 21, "per_patch", 0, 0, 0),
    (9, 2, 17, "per_patch", 0, 0, 0),
    (6, 3, 9, "per_patch", 0, 0, 0),
    (16, 2, 33, "staged", 0, 0, 4),
    (4, 3, 14, "staged", 0, 0, 1),
]
MODES = {"pipelined": 0, "per_patch": 1, "staged": 2}


@pytest.mark.parametrize("p,dim,T,mode,chunk,slots,threads", CASES)
@pytest.mark.parametrize("periodic", [False, True])
def test_host_patches_match_oracle_and_device_path(p, dim, T, mode, chunk, slots, threads, periodic):
    from paper_2306_16731_amd import fvpatch
    _announce(f"p={p} dim={dim} T={T} mode={mode} chunk={chunk} slots={slots} threads={threads} periodic={periodic}")
    b = wl.make_uniform(T, p, dim=dim, seed=p + T, pulse=True)
    m = MODES[mode]
    src, dst, lam, stats = run_host(b, m, chunk, slots, threads, periodic)
    got = gathered(b, dst)
    # the inputs are untouched
    assert np.array_equal(gathered(b, src), b.data)
    want, want_lam = oracle.batch_update(b.data, b.sizes, b.offsets, dim, 5, 1.1e-3, wl.H_DEFAULT, wl.GAMMA,
                                         periodic)
    err = hp.component_errors(got, want, 5)
    assert np.all(err <= TOL), err
    assert hp.lambda_error(lam, want_lam) <= TOL
    dev, dev_lam = hp.gpu_step(b.data, b.sizes, b.offsets, dim, 5, 1.1e-3, wl.H_DEFAULT, wl.GAMMA, periodic)
    assert np.array_equal(got, dev), "host-memory path differs from the device path"
    assert np.array_equal(lam, dev_lam)
    n = b.data.nbytes
    assert stats["bytes_to_device"] == n
    assert stats["bytes_to_host"] == n + 8 * T
    assert stats["seconds"] > 0.0


def test_without_lambda_and_repeated_calls():
    """lambda_out NULL; the same staging serves a second, larger call and a third
    with another patch size (buffers grow) with the results still exact."""
    from paper_2306_16731_amd import fvpatch
    for (p, dim, T, chunk) in [(16, 2, 12, 3), (16, 2, 40, 7), (8, 3, 30, 4), (3, 2, 9, 2)]:
        _announce(f"repeated p={p} dim={dim} T={T} chunk={chunk}")
        b = wl.make_uniform(T, p, dim=dim, seed=T)
        src, dst, lam, stats = run_host(b, fvpatch.FV_TRANSFER_PIPELINED, chunk, 2, 3, want_lambda=False)
        dev, _ = hp.gpu_step(b.data, b.sizes, b.offsets, dim, 5, 1.1e-3, wl.H_DEFAULT, wl.GAMMA, False)
        assert np.array_equal(gathered(b, dst), dev)
        assert stats["bytes_to_host"] == b.data.nbytes


def test_patches_in_one_array_at_gaps():
    """Host patches that are views into one larger array at uneven gaps (odd double
    offsets: staging copies must not assume alignment); the gaps are not written."""
    from paper_2306_16731_amd import fvpatch
    _announce("views at gaps")
    p, dim, T = 16, 2, 13
    b = wl.make_uniform(T, p, dim=dim, seed=3)
    n = (p + 2) ** dim * 5
    rng = np.random.Generator(np.random.PCG64(8))
    starts = np.cumsum(np.concatenate([[1], n + rng.integers(1, 5, size=T - 1)]))
    big_in = rng.uniform(-1, 1, int(starts[-1] + n + 3))
    big_out = np.full_like(big_in, 7.0)
    for t in range(T):
        big_in[starts[t]:starts[t] + n] = b.data[b.offsets[t]:b.offsets[t] + n]
    src = [big_in[s:s + n] for s in starts]
    dst = [big_out[s:s + n] for s in starts]
    lam = np.zeros(T)
    fvpatch.fv_host_patches_update(src, dst, b.sizes, T, dim, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, 0, lam,
                                   config={"chunk_bytes": 3 * 8 * n, "slots": 2})
    dev, dev_lam = hp.gpu_step(b.data, b.sizes, b.offsets, dim, 5, 1e-3, wl.H_DEFAULT, wl.GAMMA, False)
    assert np.array_equal(np.concatenate(dst), dev)
    assert np.array_equal(lam, dev_lam)
    inside = np.zeros(big_out.size, bool)
    for s in starts:
        inside[s:s + n] = True
    assert np.all(big_out[~inside] == 7.0), "wrote between the patches"


def test_empty_and_single():
    from paper_2306_16731_amd import fvpatch
    _announce("empty and single")
    assert fvpatch.fv_host_patches_update([], [], None, 0, 2, 5, 1e-3, 0.1, 1.4) == fvpatch.FV_OK
    b = wl.make_uniform(1, 17, dim=2, seed=1)
    for mode in (fvpatch.FV_TRANSFER_PIPELINED, fvpatch.FV_TRANSFER_PER_PATCH, fvpatch.FV_TRANSFER_STAGED):
        src, dst, lam, _ = run_host(b, mode)
        want, want_lam = oracle.batch_update(b.data, b.sizes, b.offsets, 2, 5, 1.1e-3, wl.H_DEFAULT, wl.GAMMA)
        assert inv.rel_err(dst[0], want) <= TOL
        assert abs(lam[0] - want_lam[0]) <= TOL * want_lam[0]


def pinned_patches(batch, gaps=False, seed=0):
    """The batch's patches as views into two pinned arenas from fv_host_alloc (inputs filled,
    outputs NaN), in a shuffled order, optionally at uneven (odd double) gaps."""
    from paper_2306_16731_amd import fvpatch
    T = batch.num_patches
    n = int((int(batch.sizes[0]) + 2) ** batch.dim * batch.nq)
    rng = np.random.Generator(np.random.PCG64(seed))
    step = n + (3 if gaps else 0)
    total = T * step + 8
    a_in = fvpatch.fv_host_alloc(8 * total)
    a_out = fvpatch.fv_host_alloc(8 * total)
    big_in = fvpatch.pinned_array(a_in, total)
    big_out = fvpatch.pinned_array(a_out, total)
    big_in[:] = 0.0
    big_out[:] = np.nan
    place = rng.permutation(T)
    shift = 1 if gaps else 0
    src = [big_in[shift + place[t] * step: shift + place[t] * step + n] for t in range(T)]
    dst = [big_out[shift + place[t] * step: shift + place[t] * step + n] for t in range(T)]
    for t in range(T):
        src[t][:] = batch.data[batch.offsets[t]:batch.offsets[t] + n]
    return (a_in, a_out), src, dst


ZERO_COPY_CASES = [  # (p, dim, T, chunk patches, slots, gaps, periodic)
    (16, 2, 37, 5, 3, False, True),
    (16, 2, 29, 0, 0, True, False),     # odd double offsets: 8-byte moves; defaults (one chunk)
    (7, 2, 23, 4, 1, False, False),     # one slot: chunks in turn
    (8, 3, 19, 3, 4, False, True),
    (5, 3, 11, 2, 8, True, False),
]


@pytest.mark.parametrize("p,dim,T,chunk,slots,gaps,periodic", ZERO_COPY_CASES)
def test_zero_copy_matches_device_path(p, dim, T, chunk, slots, gaps, periodic):
    from paper_2306_16731_amd import fvpatch
    _announce(f"zero copy p={p} dim={dim} T={T} chunk={chunk} slots={slots} gaps={gaps} periodic={periodic}")
    b = wl.make_uniform(T, p, dim=dim, seed=p + 2 * T, pulse=True)
    arenas, src, dst = pinned_patches(b, gaps=gaps, seed=T)
    try:
        lam = np.full(T, -1.0)
        pbytes = src[0].nbytes
        cfg = {"mode": fvpatch.FV_TRANSFER_ZERO_COPY, "slots": slots,
               "chunk_bytes": int(pbytes * chunk + pbytes // 2) if chunk else 0}
        stats = {}
        fvpatch.fv_host_patches_update(src, dst, b.sizes, T, dim, 5, 1.1e-3, wl.H_DEFAULT, wl.GAMMA,
                                       fvpatch.FV_HALO_PERIODIC if periodic else 0, lam, config=cfg, stats=stats)
        got = np.concatenate([d.copy() for d in dst])
        dev, dev_lam = hp.gpu_step(b.data, b.sizes, b.offsets, dim, 5, 1.1e-3, wl.H_DEFAULT, wl.GAMMA, periodic)
        assert np.array_equal(got, dev), "zero-copy path differs from the device path"
        assert np.array_equal(lam, dev_lam)
        assert np.array_equal(np.concatenate([s.copy() for s in src]), b.data), "inputs changed"
        assert stats["bytes_to_device"] == b.data.nbytes and stats["host_copy_seconds"] == 0.0
    finally:
        del src, dst
        for a in arenas:
            fvpatch.fv_host_free(a)


def test_zero_copy_refuses_pageable_patches():
    from paper_2306_16731_amd import fvpatch
    _announce("zero copy refuses pageable memory")
    b = wl.make_uniform(4, 6, dim=2, seed=2)
    arenas, src, dst = pinned_patches(b)
    try:
        pageable = [np.zeros_like(d) for d in dst]
        mixed = list(src[:3]) + [b.data[b.offsets[3]:b.offsets[3] + src[3].size].copy()]
        cfg = {"mode": fvpatch.FV_TRANSFER_ZERO_COPY}
        assert fvpatch.fv_host_patches_update(src, pageable, b.sizes, 4, 2, 5, 1e-3, 0.1, 1.4, config=cfg,
                                              raise_on_error=False) == fvpatch.FV_ERR_INVALID_ARG
        assert fvpatch.fv_host_patches_update(mixed, dst, b.sizes, 4, 2, 5, 1e-3, 0.1, 1.4, config=cfg,
                                              raise_on_error=False) == fvpatch.FV_ERR_INVALID_ARG
        # a patch that runs past the end of its pinned block
        a = fvpatch.fv_host_alloc(8 * 100)
        try:
            short = [fvpatch.pinned_array(a, 100)] * 1
            assert fvpatch.fv_host_patches_update(short, dst[:1], b.sizes[:1], 1, 2, 5, 1e-3, 0.1, 1.4, config=cfg,
                                                  raise_on_error=False) == fvpatch.FV_ERR_INVALID_ARG
        finally:
            del short
            fvpatch.fv_host_free(a)
        assert fvpatch.fv_host_free(a, raise_on_error=False) == fvpatch.FV_ERR_INVALID_ARG   # freed already
    finally:
        del src, dst
        for x in arenas:
            fvpatch.fv_host_free(x)
