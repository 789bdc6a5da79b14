"""The C-ABI library on the host (no GPU): it loads, exports every declared
symbol, and rejects every invalid argument before touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2306_16731_amd import build as fvbuild
from paper_2306_16731_amd import fvpatch as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Fake device addresses: validation never dereferences them.
IN = 0x10000000
OUT = 0x20000000
LAM = 0x30000000


@pytest.fixture(scope="module", autouse=True)
def built():
    if fvbuild.stale():
        fvbuild.build()
    F.load()


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "fvpatch.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(fv_[a-z0-9_]+)\s*\(", hdr)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(F.LIBRARY)
    names = declared_functions()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/fvpatch.h but not exported"
    assert sorted(F.EXPORTS) == names, "binding's EXPORTS list out of date with the header"


def test_header_constants_match_binding():
    hdr = open(os.path.join(ROOT, "include", "fvpatch.h")).read()
    for name in ["FV_MAX_P_2D", "FV_MAX_P_3D", "FV_NOALLOC_MAX_PATCHES"]:
        assert int(re.search(rf"#define {name} (\d+)", hdr).group(1)) == getattr(F, name)
    assert 1 << int(re.search(r"#define FV_MAX_OFFSET \(1LL << (\d+)\)", hdr).group(1)) == F.FV_MAX_OFFSET
    for name in ["FV_HALO_PERIODIC", "FV_HALO_FROM_IN", "FV_PLAN_NO_PERSIST", "FV_PLAN_PER_CLASS"]:
        assert int(re.search(rf"#define {name} (0x[0-9a-f]+)u", hdr).group(1), 16) == getattr(F, name), name
    for name in ["FV_KERNEL_AUTO", "FV_KERNEL_BLOCK", "FV_KERNEL_WAVE", "FV_KERNEL_TILE", "FV_KERNEL_FIXED"]:
        assert int(re.search(rf"#define {name} (\d+)", hdr).group(1)) == getattr(F, name), name
    found = re.findall(r"p in \{([0-9, ]+)\}", hdr)
    assert tuple(int(x) for x in found[0].split(",")) == F.FIXED_SIZES_2D
    assert tuple(int(x) for x in found[1].split(",")) == F.FIXED_SIZES_3D


def call(**kw):
    args = dict(patches_in=IN, patches_out=OUT, sizes=[4] * 3, offsets=None, num_patches=3, dim=2, unknowns=5,
                dt=1e-3, h=1 / 48, gamma=1.4, flags=0, lambda_out=LAM, stream=0)
    args.update(kw)
    return F.fv_patch_batch_update(raise_on_error=False, **args)


def test_build_id_is_the_hash_of_the_sources():
    """The loaded library reports the hash of the sources it was built from, and the loader refuses
    a library whose id differs from the sources beside it."""
    assert F.load().fv_build_id().decode() == fvbuild.source_hash()
    assert fvbuild.stale() is False


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures and numpy record types have the header's sizes and field
    offsets (a C program compiled against include/fvpatch.h prints them)."""
    import subprocess
    structs = {"fv_tuning": F.fv_tuning, "fv_plan_stats": F.fv_plan_stats, "fv_server_config": F.fv_server_config,
               "fv_serve_request": F.fv_serve_request, "fv_server_stats": F.fv_server_stats,
               "fv_transfer_config": F.fv_transfer_config, "fv_transfer_stats": F.fv_transfer_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fvpatch.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    for fname in F.BATCH_RECORD_DTYPE.names:
        lines.append(f'printf("fv_batch_record.{fname} %zu\\n", offsetof(fv_batch_record, {fname}));')
    lines.append('printf("fv_batch_record %zu\\n", sizeof(fv_batch_record));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.split("\n") if line)
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)
    assert int(got["fv_batch_record"]) == F.BATCH_RECORD_DTYPE.itemsize
    for fname in F.BATCH_RECORD_DTYPE.names:
        assert int(got[f"fv_batch_record.{fname}"]) == F.BATCH_RECORD_DTYPE.fields[fname][1], fname


def test_server_config_validation():
    """fv_server_create rejects bad configurations before touching a device."""
    for kw in (dict(max_retries=-1), dict(max_retries=17), dict(deadline_ms=-1.0), dict(deadline_ms=float("nan")),
               dict(max_inflight=2000), dict(mode=7), dict(gamma=1.0), dict(flags=0x80)):
        args = dict(budget_bytes=1 << 30)
        args.update(kw)
        st, h = F.fv_server_create(raise_on_error=False, **args)
        assert st == F.FV_ERR_INVALID_ARG, kw
    st, h = F.fv_server_create(0, raise_on_error=False)
    assert st == F.FV_ERR_INVALID_ARG


def test_status_strings():
    assert F.fv_status_string(F.FV_OK) == "ok"
    assert F.fv_status_string(F.FV_ERR_OVERLAP) == "overlapping buffers"
    assert F.fv_version() >= 100


INVALID_CALLS = [
    (dict(dim=1), F.FV_ERR_INVALID_ARG),
    (dict(dim=4), F.FV_ERR_INVALID_ARG),
    (dict(unknowns=3), F.FV_ERR_INVALID_ARG),
    (dict(dim=3, unknowns=4), F.FV_ERR_UNSUPPORTED),
    (dict(dt=0.0), F.FV_ERR_INVALID_ARG),
    (dict(dt=-1e-3), F.FV_ERR_INVALID_ARG),
    (dict(dt=float("nan")), F.FV_ERR_INVALID_ARG),
    (dict(dt=float("inf")), F.FV_ERR_INVALID_ARG),
    (dict(h=0.0), F.FV_ERR_INVALID_ARG),
    (dict(h=float("nan")), F.FV_ERR_INVALID_ARG),
    (dict(gamma=1.0), F.FV_ERR_INVALID_ARG),
    (dict(gamma=float("nan")), F.FV_ERR_INVALID_ARG),
    (dict(flags=0x8), F.FV_ERR_INVALID_ARG),
    (dict(num_patches=-1), F.FV_ERR_INVALID_ARG),
    (dict(patches_in=0), F.FV_ERR_INVALID_ARG),
    (dict(patches_out=0), F.FV_ERR_INVALID_ARG),
    (dict(sizes=None), F.FV_ERR_INVALID_ARG),
    (dict(patches_in=IN + 4), F.FV_ERR_INVALID_ARG),
    (dict(lambda_out=LAM + 2), F.FV_ERR_INVALID_ARG),
    (dict(sizes=[0, 4, 4]), F.FV_ERR_INVALID_ARG),
    (dict(sizes=[4, 65, 4]), F.FV_ERR_INVALID_ARG),
    (dict(dim=3, sizes=[25, 4, 4]), F.FV_ERR_INVALID_ARG),
    (dict(sizes=[4, 5, 4]), F.FV_ERR_INVALID_ARG),           # offsets NULL needs equal sizes
    (dict(offsets=[0, -5, 200]), F.FV_ERR_INVALID_ARG),
    (dict(offsets=[0, 1 << 62, 200]), F.FV_ERR_INVALID_ARG),   # beyond FV_MAX_OFFSET
    (dict(offsets=[0, (1 << 48) - 100, 200]), F.FV_ERR_INVALID_ARG),
    (dict(offsets=[0, 100, 400]), F.FV_ERR_OVERLAP),         # patch 0 spans 180 doubles
    (dict(offsets=[400, 0, 100]), F.FV_ERR_OVERLAP),         # unsorted and overlapping
    (dict(patches_out=IN + 8 * 100), F.FV_ERR_OVERLAP),      # in and out overlap
    (dict(patches_out=IN), F.FV_ERR_OVERLAP),
    (dict(lambda_out=OUT + 8), F.FV_ERR_OVERLAP),
]


@pytest.mark.parametrize("kw,status", INVALID_CALLS)
def test_invalid_arguments_rejected_before_device(kw, status):
    st = call(**kw)
    assert st == status, (st, F.fv_last_error())
    assert F.fv_last_error() != ""


def call_noalloc(**kw):
    args = dict(patches_in=IN, patches_out=OUT, sizes=[4] * 3, offsets=None, num_patches=3, dim=2, unknowns=5,
                dt=1e-3, h=1 / 48, gamma=1.4, flags=0, lambda_out=LAM, stream=0)
    args.update(kw)
    return F.fv_patch_batch_update_noalloc(raise_on_error=False, **args)


@pytest.mark.parametrize("kw,status", INVALID_CALLS)
def test_noalloc_rejects_the_same_arguments_before_device(kw, status):
    st = call_noalloc(**kw)
    assert st == status, (st, F.fv_last_error())
    assert F.fv_last_error() != ""


def test_noalloc_limits_and_no_device():
    """More patches than the fixed descriptor array holds is an argument error, raised before
    anything else is looked at; valid calls reach the device check."""
    T = F.FV_NOALLOC_MAX_PATCHES + 1
    assert call_noalloc(num_patches=T, sizes=np.full(T, 4, np.int32)) == F.FV_ERR_INVALID_ARG
    assert str(F.FV_NOALLOC_MAX_PATCHES) in F.fv_last_error()
    assert call_noalloc(num_patches=0, sizes=None, patches_in=0, patches_out=0) == F.FV_OK
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    assert call_noalloc() == F.FV_ERR_NO_DEVICE
    assert call_noalloc(offsets=[360, 0, 180]) == F.FV_ERR_NO_DEVICE
    T = F.FV_NOALLOC_MAX_PATCHES
    sizes = np.full(T, 2, np.int32)
    offs = (np.arange(T, dtype=np.int64)[::-1] * 80).copy()  # unsorted: checked in the fixed sort array
    assert call_noalloc(num_patches=T, sizes=sizes, offsets=offs) == F.FV_ERR_NO_DEVICE


def test_zero_patches_is_a_noop():
    assert call(num_patches=0, sizes=None, patches_in=0, patches_out=0) == F.FV_OK
    assert F.fv_last_error() == ""


def test_valid_arguments_without_a_gpu_report_no_device():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    assert call() == F.FV_ERR_NO_DEVICE
    assert call(offsets=[0, 180, 360]) == F.FV_ERR_NO_DEVICE
    assert call(offsets=[360, 0, 180]) == F.FV_ERR_NO_DEVICE      # unsorted, disjoint
    assert call(lambda_out=None) == F.FV_ERR_NO_DEVICE
    assert call(flags=F.FV_HALO_FROM_IN) == F.FV_ERR_NO_DEVICE       # a valid flag: fails only for want of a GPU
    assert call(flags=F.FV_HALO_FROM_IN | F.FV_HALO_PERIODIC) == F.FV_ERR_NO_DEVICE
    st, h = F.fv_plan_create([4, 4], None, 2, 2, 5, F.FV_HALO_FROM_IN | F.FV_PLAN_PER_CLASS, raise_on_error=False)
    assert st == F.FV_ERR_NO_DEVICE and not h


def _expected_status(sizes, offsets, out, lam, dim=2, nq=5):
    """Brute-force model of the layout and buffer checks: every patch range, every pair."""
    if any(o < 0 or o + (p + 2) ** dim * nq > F.FV_MAX_OFFSET for p, o in zip(sizes, offsets)):
        return F.FV_ERR_INVALID_ARG
    ranges = [(o, o + (p + 2) ** dim * nq) for p, o in zip(sizes, offsets)]
    for a in range(len(ranges)):
        for b in range(a + 1, len(ranges)):
            if ranges[a][0] < ranges[b][1] and ranges[b][0] < ranges[a][1]:
                return F.FV_ERR_OVERLAP
    lo, hi = min(r[0] for r in ranges), max(r[1] for r in ranges)
    spans = {"in": (IN + 8 * lo, IN + 8 * hi), "out": (out + 8 * lo, out + 8 * hi)}
    if spans["in"][0] < spans["out"][1] and spans["out"][0] < spans["in"][1]:
        return F.FV_ERR_OVERLAP
    if lam is not None:
        l0, l1 = lam, lam + 8 * len(sizes)
        if any(l0 < b and a < l1 for a, b in spans.values()):
            return F.FV_ERR_OVERLAP
    return F.FV_ERR_NO_DEVICE


def test_layout_checks_match_a_brute_force_model():
    """Random batches (gapped, shuffled, overlapping, out of range) and buffer placements: the library's
    verdict before any device work equals the pairwise check's."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible: a valid call would launch on the fake addresses")
    except ImportError:
        pass
    from hypothesis import given, settings, strategies as stg

    big = stg.sampled_from([-1, F.FV_MAX_OFFSET - 500, F.FV_MAX_OFFSET - 100, F.FV_MAX_OFFSET, 1 << 62])

    @stg.composite
    def batches(draw):
        T = draw(stg.integers(1, 12))
        sizes = draw(stg.lists(stg.integers(1, 9), min_size=T, max_size=T))
        gap = stg.one_of(*[stg.integers(0, 60)] * 7, stg.integers(-150, -1))
        gaps = draw(stg.lists(gap, min_size=T, max_size=T))
        offsets, pos = [], 0
        for p, g in zip(sizes, gaps):
            pos = max(0, pos + g)
            offsets.append(pos)
            pos += (p + 2) ** 2 * 5
        offsets = draw(stg.permutations(offsets))
        if draw(stg.integers(0, 9)) == 0:
            offsets[draw(stg.integers(0, T - 1))] = draw(big)
        out = draw(stg.sampled_from([OUT] * 4 + [IN, IN + 8 * 50, IN + 8 * pos, IN + 8 * (pos - 1), IN - 8 * 300]))
        lam = draw(stg.sampled_from([None, LAM, LAM, IN, OUT + 8 * 7, IN - 8 * T, IN - 8 * (T - 1)]))
        return sizes, offsets, out, lam

    @settings(max_examples=400, deadline=None, derandomize=True)
    @given(batches())
    def check(case):
        sizes, offsets, out, lam = case
        st = call(sizes=sizes, offsets=offsets, num_patches=len(sizes), patches_out=out, lambda_out=lam)
        assert st == _expected_status(sizes, offsets, out, lam), (case, st, F.fv_last_error())

    check()


def test_error_raises_with_detail():
    with pytest.raises(F.FvError) as e:
        F.fv_patch_batch_update(IN, OUT, [4], None, 1, 5, 5, 1e-3, 1 / 48)
    assert e.value.status == F.FV_ERR_INVALID_ARG and "dim" in e.value.detail


def test_binding_has_no_compute_of_its_own():
    """The binding module holds no update arithmetic (it only marshals arguments)."""
    src = open(os.path.join(ROOT, "paper_2306_16731_amd", "fvpatch.py")).read()
    for token in ["sqrt", "gamma - 1", "0.5 *", "rusanov", "import oracle", "from oracle"]:
        assert token not in src.lower(), token


def test_plan_validation_before_device():
    """Plan creation rejects bad compositions before any device work."""
    bad = [
        (dict(sizes=[4, 4], offsets=None, num_patches=2, dim=5, unknowns=5), F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 4], offsets=None, num_patches=0, dim=2, unknowns=5), F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 5], offsets=None, num_patches=2, dim=2, unknowns=5), F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 4], offsets=[0, 10], num_patches=2, dim=2, unknowns=5), F.FV_ERR_OVERLAP),
        (dict(sizes=[4, 4], offsets=None, num_patches=2, dim=2, unknowns=5, flags=0x8), F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 4], offsets=None, num_patches=2, dim=2, unknowns=5,
              flags=F.FV_PLAN_NO_PERSIST | F.FV_PLAN_PER_CLASS), F.FV_ERR_INVALID_ARG),
    ]
    for kw, status in bad:
        st, h = F.fv_plan_create(raise_on_error=False, **kw)
        assert st == status and not h, (kw, st, F.fv_last_error())
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    st, h = F.fv_plan_create([4, 4], None, 2, 2, 5, raise_on_error=False)
    assert st == F.FV_ERR_NO_DEVICE and not h
    assert F.fv_plan_destroy(None) == F.FV_OK
    assert F.load().fv_plan_replay(None, None) == F.FV_ERR_INVALID_ARG
    assert F.load().fv_plan_execute(None, IN, OUT, 1e-3, None, 1 / 48, 1.4, None, None) == F.FV_ERR_INVALID_ARG
    assert F.load().fv_plan_get_tuning(None, 4, None) == F.FV_ERR_INVALID_ARG


def test_plan_tuning_table_validation_before_device():
    """A plan's own tuning table is checked like fv_set_tuning's argument, before any device work;
    entries for another (dim, unknowns) are ignored."""
    base = dict(sizes=[4, 4], offsets=None, num_patches=2, dim=2, unknowns=5)
    bad = [
        ({(2, 5, 4): dict(kernel=9)}, F.FV_ERR_INVALID_ARG),
        ({(2, 5, 4): dict(kernel=F.FV_KERNEL_FIXED)}, F.FV_ERR_UNSUPPORTED),       # no fixed build for p = 4
        ({(2, 5, 4): dict(kernel=F.FV_KERNEL_WAVE, block=100)}, F.FV_ERR_INVALID_ARG),
        ({(2, 5, 65): dict(kernel=F.FV_KERNEL_BLOCK)}, F.FV_ERR_INVALID_ARG),
        ([(2, 5, 4, dict(kernel=F.FV_KERNEL_WAVE)), (2, 5, 4, dict(kernel=F.FV_KERNEL_BLOCK))], F.FV_ERR_INVALID_ARG),
    ]
    for tune, status in bad:
        st, h = F.fv_plan_create(raise_on_error=False, tune=tune, **base)
        assert st == status and not h, (tune, st, F.fv_last_error())
    # an entry for another dimension is ignored: the call gets as far as the device check
    st, h = F.fv_plan_create(raise_on_error=False, tune={(3, 5, 99): dict(kernel=9)}, **base)
    try:
        import torch
        expect = F.FV_OK if torch.cuda.is_available() else F.FV_ERR_NO_DEVICE
    except ImportError:
        expect = F.FV_ERR_NO_DEVICE
    assert st == expect, F.fv_last_error()
    if h:
        F.fv_plan_destroy(h)
    assert F.load().fv_plan_create(ctypes.byref(ctypes.c_void_p()), (ctypes.c_int32 * 2)(4, 4), None, 2, 2, 5, 0,
                                   None, 3) == F.FV_ERR_INVALID_ARG


def test_tuning_table_on_host():
    """Defaults and validation of the per-class launch parameters (no device needed)."""
    try:
        assert F.fv_get_tuning(2, 5, 16) == dict(kernel=F.FV_KERNEL_FIXED, block=64, prefetch=2, rows=12)
        for p in F.FIXED_SIZES_2D:
            assert F.fv_get_tuning(2, 5, p)["kernel"] == F.FV_KERNEL_FIXED
        assert F.fv_get_tuning(2, 4, 16)["kernel"] == F.FV_KERNEL_WAVE     # no fixed build for four unknowns
        assert F.fv_get_tuning(2, 5, 7)["kernel"] == F.FV_KERNEL_WAVE
        assert F.fv_get_tuning(3, 5, 7)["kernel"] == F.FV_KERNEL_BLOCK
        for p in F.FIXED_SIZES_3D:
            assert F.fv_get_tuning(3, 5, p) == dict(kernel=F.FV_KERNEL_FIXED, block=64, prefetch=2, rows=2)
        bad = [
            ((2, 4, 16, dict(kernel=4, block=0, prefetch=0, rows=0)), F.FV_ERR_UNSUPPORTED),
            ((2, 5, 7, dict(kernel=4, block=0, prefetch=0, rows=0)), F.FV_ERR_UNSUPPORTED),
            ((3, 5, 7, dict(kernel=4, block=0, prefetch=0, rows=0)), F.FV_ERR_UNSUPPORTED),
            ((3, 5, 10, dict(kernel=4, block=0, prefetch=0, rows=0)), F.FV_ERR_UNSUPPORTED),
            ((2, 5, 16, dict(kernel=4, block=256, prefetch=0, rows=0)), F.FV_ERR_INVALID_ARG),
            ((2, 5, 16, dict(kernel=4, block=0, prefetch=3, rows=0)), F.FV_ERR_INVALID_ARG),
            ((2, 5, 16, dict(kernel=4, block=0, prefetch=0, rows=5)), F.FV_ERR_INVALID_ARG),
            ((2, 5, 16, dict(kernel=5, block=0, prefetch=0, rows=0)), F.FV_ERR_INVALID_ARG),
        ]
        for (dim, nq, p, t), status in bad:
            assert F.fv_set_tuning(dim, nq, p, t, raise_on_error=False) == status, (dim, nq, p, t)
        # the build's own values are accepted; automatic choice with other values falls back to the wave kernel
        assert F.fv_set_tuning(2, 5, 16, dict(kernel=4, block=64, prefetch=2, rows=12), raise_on_error=False) == F.FV_OK
        assert F.fv_set_tuning(2, 5, 16, dict(kernel=0, block=0, prefetch=4, rows=6), raise_on_error=False) == F.FV_OK
        assert F.fv_get_tuning(2, 5, 16) == dict(kernel=F.FV_KERNEL_WAVE, block=256, prefetch=4, rows=6)
        assert F.fv_set_tuning(3, 5, 8, dict(kernel=4, block=64, prefetch=2, rows=2), raise_on_error=False) == F.FV_OK
    finally:
        for p in F.FIXED_SIZES_2D:
            F.fv_set_tuning(2, 5, p, None)
        for p in F.FIXED_SIZES_3D:
            F.fv_set_tuning(3, 5, p, None)


def test_mesh_validation_before_device():
    """Mesh creation and the mesh calls reject bad arguments before any device work."""
    nb_ok = [[-1, -1, -1, -1]] * 2
    bad = [
        (dict(sizes=[4, 4], offsets=None, neighbors=nb_ok, num_patches=2, dim=4, unknowns=5), F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 4], offsets=None, neighbors=nb_ok, num_patches=0, dim=2, unknowns=5), F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 4], offsets=None, neighbors=None, num_patches=2, dim=2, unknowns=5), F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 5], offsets=[0, 1000], neighbors=nb_ok, num_patches=2, dim=2, unknowns=5),
         F.FV_ERR_UNSUPPORTED),
        (dict(sizes=[4, 4], offsets=None, neighbors=[[2, -1, -1, -1], [-1] * 4], num_patches=2, dim=2, unknowns=5),
         F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 4], offsets=None, neighbors=[[-2, -1, -1, -1], [-1] * 4], num_patches=2, dim=2, unknowns=5),
         F.FV_ERR_INVALID_ARG),
        (dict(sizes=[4, 4], offsets=[0, 10], neighbors=nb_ok, num_patches=2, dim=2, unknowns=5), F.FV_ERR_OVERLAP),
    ]
    for kw, status in bad:
        st, h = F.fv_mesh_create(raise_on_error=False, **kw)
        assert st == status and not h, (kw, st, F.fv_last_error())
    lib = F.load()
    assert lib.fv_mesh_halo_fill(None, IN, None) == F.FV_ERR_INVALID_ARG
    assert lib.fv_mesh_step(None, IN, OUT, LAM, LAM, 1.4, None, None) == F.FV_ERR_INVALID_ARG
    assert F.fv_mesh_destroy(None) == F.FV_OK
    assert lib.fv_local_dt(LAM, LAM, 0, 2, 0.4, OUT, None) == F.FV_OK
    assert lib.fv_local_dt(LAM, LAM, 4, 5, 0.4, OUT, None) == F.FV_ERR_INVALID_ARG
    assert lib.fv_local_dt(LAM, LAM, 4, 2, 0.0, OUT, None) == F.FV_ERR_INVALID_ARG
    assert lib.fv_local_dt(None, LAM, 4, 2, 0.4, OUT, None) == F.FV_ERR_INVALID_ARG
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    st, h = F.fv_mesh_create([4, 4], None, nb_ok, 2, 2, 5, raise_on_error=False)
    assert st == F.FV_ERR_NO_DEVICE and not h


def test_flavour_validation_before_device():
    kw = dict(patches_in=IN, patches_out=OUT, sizes=[4] * 3, offsets=None, num_patches=3, dim=2, unknowns=5,
              dt=1e-3, h=1 / 48, gamma=1.4, flags=0, lambda_out=LAM, stream=0)

    def call(flavour, **over):
        a = dict(kw)
        a.update(over)
        return F.fv_flavour_update(flavour, raise_on_error=False, **a)

    assert call(0) == F.FV_ERR_INVALID_ARG
    assert call(4) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_FLAVOUR_BATCHED, unknowns=4) == F.FV_ERR_UNSUPPORTED
    assert call(F.FV_FLAVOUR_BATCHED, sizes=[4, 5, 4], offsets=[0, 200, 500]) == F.FV_ERR_UNSUPPORTED
    assert call(F.FV_FLAVOUR_PATCH_WISE, dim=3, sizes=[9] * 3) == F.FV_ERR_UNSUPPORTED   # 729 interior volumes
    assert call(F.FV_FLAVOUR_TASK_GRAPH, dt=-1.0) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_FLAVOUR_TASK_GRAPH, patches_out=IN) == F.FV_ERR_OVERLAP
    assert call(F.FV_FLAVOUR_BATCHED, num_patches=0, sizes=None, patches_in=0, patches_out=0) == F.FV_OK
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    assert call(F.FV_FLAVOUR_BATCHED) == F.FV_ERR_NO_DEVICE


def test_host_patches_validation_before_device():
    """fv_host_patches_update checks its arguments on the host before it touches a device."""
    p, T = 4, 3
    n = (p + 2) ** 2 * 5
    src = [np.zeros(n) for _ in range(T)]
    dst = [np.zeros(n) for _ in range(T)]
    lam = np.zeros(T)
    kw = dict(patches_in=src, patches_out=dst, sizes=[p] * T, num_patches=T, dim=2, unknowns=5, dt=1e-3, h=1 / 48,
              gamma=1.4, flags=0, lambda_out=lam)

    def call(**over):
        a = dict(kw)
        a.update(over)
        return F.fv_host_patches_update(raise_on_error=False, **a)

    assert call(dt=-1.0) == F.FV_ERR_INVALID_ARG
    assert call(dim=4) == F.FV_ERR_INVALID_ARG
    assert call(sizes=[p, p + 1, p]) == F.FV_ERR_UNSUPPORTED
    assert call(sizes=[0] * T) == F.FV_ERR_INVALID_ARG
    assert call(config={"mode": 3}) == F.FV_ERR_INVALID_ARG
    assert call(config={"slots": F.FV_TRANSFER_MAX_SLOTS + 1}) == F.FV_ERR_INVALID_ARG
    assert call(config={"host_threads": -1}) == F.FV_ERR_INVALID_ARG
    assert call(config={"chunk_bytes": 8 * n - 8}) == F.FV_ERR_INVALID_ARG   # below one patch
    assert call(patches_out=[dst[0], src[1], dst[2]]) == F.FV_ERR_OVERLAP     # an output is an input
    assert call(patches_out=[dst[0], dst[0], dst[2]]) == F.FV_ERR_OVERLAP     # two outputs share an array
    big = np.zeros(2 * n)
    half = np.array([big.ctypes.data, big.ctypes.data + 8 * (n // 2), dst[2].ctypes.data], np.uintp)
    assert call(patches_out=half) == F.FV_ERR_OVERLAP                         # outputs overlap in part
    assert call(patches_in=np.array([src[0].ctypes.data, 0, src[2].ctypes.data], np.uintp)) == F.FV_ERR_INVALID_ARG
    assert call(num_patches=0, sizes=None, patches_in=[], patches_out=[]) == F.FV_OK
    with pytest.raises(ValueError):
        call(patches_in=[np.zeros(n, np.float32)] * T)
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    assert call() == F.FV_ERR_NO_DEVICE


def test_host_patches_alignment():
    n = (4 + 2) ** 2 * 5
    raw = np.zeros(3 * n + 1)
    src = [np.zeros(n) for _ in range(2)]
    odd = np.array([raw.ctypes.data + 4, raw.ctypes.data + 8 * n + 8], np.uintp)   # 4 bytes off
    assert F.fv_host_patches_update(src, odd, [4, 4], 2, 2, 5, 1e-3, 0.1, 1.4,
                                    raise_on_error=False) == F.FV_ERR_INVALID_ARG


def test_pde_shapes_and_validation_before_device():
    assert F.fv_pde_unknowns(F.FV_PDE_EULER, 3) == (5, 1)
    assert F.fv_pde_unknowns(F.FV_PDE_SHALLOW_WATER, 2) == (4, 2)
    assert F.fv_pde_unknowns(F.FV_PDE_ADVECTION, 3) == (1, 3)
    assert F.fv_pde_unknowns(F.FV_PDE_ACOUSTICS, 2) == (3, 2)
    assert F.fv_pde_unknowns(F.FV_PDE_ACOUSTICS_NCP, 3) == (4, 2)
    with pytest.raises(F.FvError):
        F.fv_pde_unknowns(F.FV_PDE_SHALLOW_WATER, 3)
    with pytest.raises(F.FvError):
        F.fv_pde_unknowns(5, 2)

    def call(pde, prm, dim=2, n=1, **kw):
        a = dict(patches_in=IN, patches_out=OUT, sizes=[4] * n, offsets=None, num_patches=n, dim=dim, dt=1e-3,
                 h=0.1, lambda_out=None, stream=0)
        a.update(kw)
        return F.fv_pde_batch_update(pde, prm, raise_on_error=False, **a)

    assert call(F.FV_PDE_SHALLOW_WATER, [9.81, 0.0], dim=3) == F.FV_ERR_UNSUPPORTED
    assert call(F.FV_PDE_SHALLOW_WATER, [9.81, 0.0, 1.0]) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_PDE_SHALLOW_WATER, [0.0, 0.0]) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_PDE_ACOUSTICS, [1.0, -2.0]) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_PDE_ADVECTION, [1.0, 0.0, np.inf]) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_PDE_ADVECTION, [1.0, 0.0, 0.0], dt=0.0) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_PDE_ADVECTION, [1.0, 0.0, 0.0], flags=8) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_PDE_ADVECTION, [1.0, 0.0, 0.0], patches_out=IN) == F.FV_ERR_OVERLAP
    assert call(F.FV_PDE_ADVECTION, [1.0, 0.0, 0.0], sizes=[0]) == F.FV_ERR_INVALID_ARG
    assert call(F.FV_PDE_ADVECTION, [1.0, 0.0, 0.0], n=0, sizes=None) == F.FV_OK
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    assert call(F.FV_PDE_ADVECTION, [1.0, 0.0, 0.0]) == F.FV_ERR_NO_DEVICE


def test_zero_copy_and_pinned_validation_before_device():
    n = (4 + 2) ** 2 * 5
    src = [np.zeros(n) for _ in range(2)]
    dst = [np.zeros(n) for _ in range(2)]
    # pageable patches are refused by the zero-copy mode before any device work
    assert F.fv_host_patches_update(src, dst, [4, 4], 2, 2, 5, 1e-3, 0.1, 1.4,
                                    config={"mode": F.FV_TRANSFER_ZERO_COPY},
                                    raise_on_error=False) == F.FV_ERR_INVALID_ARG
    assert F.fv_host_free(None) == F.FV_OK
    assert F.fv_host_free(src[0].ctypes.data, raise_on_error=False) == F.FV_ERR_INVALID_ARG
    assert F.fv_host_alloc(0, raise_on_error=False)[0] == F.FV_ERR_INVALID_ARG
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    assert F.fv_host_alloc(1024, raise_on_error=False)[0] == F.FV_ERR_NO_DEVICE
