"""Build the gfx950 shared library ``libfvpatch.so`` in-tree with hipcc.

    python -m paper_2306_16731_amd.build        # or call build()

The library exports the C ABI of include/fvpatch.h.  It is compiled for
gfx950 only, with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBRARY = os.path.join(PKG, "libfvpatch.so")

SOURCES = ["fv_update.hip", "fv_update2d.hip", "fv_update2d_tile.hip", "fv_step.hip", "fv_abi.hip", "fv_plan.hip", "fv_serve.hip"]
HEADERS = ["fv_internal.h", "fv_host.h", "fv_physics.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-variable",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the library needs ROCm's hipcc to build")
    return path


def build(verbose: bool = False, extra_flags: list[str] | None = None, output: str = LIBRARY) -> str:
    """Compile every source into the shared library (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [hipcc(), *HIPCC_FLAGS, *(extra_flags or []), "-I", INCLUDE, "-I", CSRC, "-o", output + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(output + ".tmp", output)
    return output


def stale() -> bool:
    """True when the library is missing or older than any source or header."""
    if not os.path.exists(LIBRARY):
        return True
    t = os.path.getmtime(LIBRARY)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(INCLUDE, "fvpatch.h")]
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose=True))
