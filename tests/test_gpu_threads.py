"""Calls of the plain entry point from several host threads at once, each thread on its own stream and
buffers, more threads than the library keeps pinned descriptor slots, with batches that grow from call to
call (so slots are reallocated while other threads' calls use theirs).  Every thread's results equal the
same sequence of calls made alone, bit for bit."""
from __future__ import annotations

import sys
import threading

import numpy as np
import pytest

from paper_2306_16731_amd import fvpatch as fv
from paper_2306_16731_amd import workloads as wl
from tests import hip_path as hp

pytestmark = pytest.mark.gpu

THREADS = 12
CALLS = 6


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fv.load()


def case(w):
    """Thread w's batch: mixed sizes at shuffled, gapped offsets (the descriptor path), and how many of its
    patches each call updates (growing)."""
    rng = np.random.Generator(np.random.PCG64(300 + w))
    T = 600 + 900 * (w % 4)
    sizes = rng.choice(np.array([3, 5, 9, 17], np.int32), size=T)
    vols = (sizes.astype(np.int64) + 2) ** 2 * 5
    gaps = rng.integers(0, 4, size=T)
    starts = np.cumsum(np.concatenate([[0], (vols + gaps)[:-1]])).astype(np.int64)
    compact = wl.make_batch(sizes, 2, 5, seed=400 + w)
    data = np.zeros(int(starts[-1] + vols[-1]), np.float64)
    for t in range(T):
        data[starts[t]:starts[t] + vols[t]] = compact.data[compact.offsets[t]:compact.offsets[t] + vols[t]]
    perm = rng.permutation(T)
    counts = [max(1, T * (c + 1) // CALLS) for c in range(CALLS)]
    flags = fv.FV_HALO_PERIODIC if w % 3 == 0 else 0
    return data, sizes[perm], starts[perm], counts, flags


def run_sequence(data, sizes, offsets, counts, flags, stream):
    """CALLS ping-pong steps on `stream`, call c over the first counts[c] patches; returns (state, lambda)."""
    t = hp.torch()
    with t.cuda.stream(stream):
        a = t.from_numpy(data).to(hp.DEVICE, non_blocking=False)
        b = a.clone()
        lam = t.zeros(len(sizes), dtype=t.float64, device=hp.DEVICE)
    stream.synchronize()
    for n in counts:
        fv.fv_patch_batch_update(a, b, sizes[:n], offsets[:n], n, 2, 5, 2e-4, wl.H_DEFAULT, wl.GAMMA, flags, lam,
                                 stream=stream)
        a, b = b, a
    stream.synchronize()
    return a.cpu().numpy(), lam.cpu().numpy()


def test_concurrent_calls_from_threads_equal_calls_alone():
    t = hp.torch()
    print(f"[gpu-threads] {THREADS} threads x {CALLS} calls, descriptor path", flush=True)
    sys.stdout.flush()
    cases = [case(w) for w in range(THREADS)]
    alone = [run_sequence(*c, t.cuda.Stream()) for c in cases]
    streams = [t.cuda.Stream() for _ in range(THREADS)]
    got = [None] * THREADS
    errors = []
    start = threading.Barrier(THREADS)

    def worker(w):
        try:
            start.wait()
            got[w] = run_sequence(*cases[w], streams[w])
        except Exception as e:  # reported below, with the thread's index
            errors.append((w, repr(e)))

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(THREADS)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not any(th.is_alive() for th in threads), "a thread did not finish"
    assert not errors, errors
    for w in range(THREADS):
        assert np.array_equal(got[w][0].view(np.int64), alone[w][0].view(np.int64)), f"state of thread {w}"
        assert np.array_equal(got[w][1].view(np.int64), alone[w][1].view(np.int64)), f"lambda of thread {w}"
