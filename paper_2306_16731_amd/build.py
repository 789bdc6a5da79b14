"""Build the gfx950 shared library ``libfvpatch.so`` in-tree with hipcc.

    python -m paper_2306_16731_amd.build        # or call build()

The library exports the C ABI of include/fvpatch.h.  It is compiled for
gfx950 only, with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import concurrent.futures
import glob
import hashlib
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBRARY = os.path.join(PKG, "libfvpatch.so")

SOURCES = ["fv_update.hip", "fv_update2d.hip", "fv_update2d_tile.hip", "fv_update3d.hip", "fv_step.hip", "fv_abi.hip",
           "fv_plan.hip", "fv_serve.hip", "fv_mesh.hip", "fv_flavours.hip",
           "fv_transfer.hip"]


def headers() -> list[str]:
    """Every header of csrc/ (all of them are included by some source)."""
    return sorted(os.path.basename(h) for h in glob.glob(os.path.join(CSRC, "*.h")))


def source_files() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES + headers()] + [os.path.join(INCLUDE, "fvpatch.h")]


def source_hash() -> str:
    """Hash of the library's sources and headers (names and contents): the build id the library
    reports through fv_build_id()."""
    h = hashlib.sha256()
    for f in source_files():
        h.update(os.path.basename(f).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wshadow",
    "-Wno-unused-variable",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the library needs ROCm's hipcc to build")
    return path


def _run(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}: {' '.join(cmd[-3:])}")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)


def build(verbose: bool = False, extra_flags: list[str] | None = None, output: str = LIBRARY) -> str:
    """Compile every source (in parallel, one object each) and link the shared
    library (always recompiles)."""
    flags = [*HIPCC_FLAGS, *(extra_flags or []), f'-DFV_BUILD_ID="{source_hash()}"', "-I", INCLUDE, "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="fvpatch_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        jobs = [[hipcc(), *flags, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1)))
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as pool:
            for f in [pool.submit(_run, j, verbose) for j in jobs]:
                f.result()
        _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", output + ".tmp", *objs], verbose)
    os.replace(output + ".tmp", output)
    return output


def stale() -> bool:
    """True when the library is missing or older than any source or header."""
    if not os.path.exists(LIBRARY):
        return True
    t = os.path.getmtime(LIBRARY)
    return any(os.path.getmtime(d) > t for d in source_files() if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose=True))
