"""The library's host code and the CPU oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU (no GPU needed).

* The library: every source is compiled host-only (device code is not built)
  with the sanitizers on the host side, and linked with a CPU stand-in of the
  HIP runtime (tests/host_sanitize/fake_hip.cpp) into a driver that calls every
  entry point of include/fvpatch.h: validation, descriptor building, plans and
  their graph capture, the comparison flavours over the benchmark's matrix
  (buffers freed between batch sizes), the serving loop with forced failures,
  meshes, transfers with host threads.  The stand-in checks launch
  configurations, that kernel pointer arguments lead into live memory, and that
  no device memory a live graph executable refers to is freed.
* The oracle: oracle/fv_oracle.c with a driver over all its entry points.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess

import pytest

from paper_2306_16731_amd import build as fvbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CLANG = "/opt/rocm/llvm/bin/clang++"
CLANG_C = "/opt/rocm/llvm/bin/clang"
SAN = ["address", "undefined"]
ENV = {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1:abort_on_error=0",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if res.returncode != 0:
        raise AssertionError(f"{' '.join(cmd[:6])} ... failed ({res.returncode}):\n{res.stdout[-4000:]}\n"
                             f"{res.stderr[-8000:]}")
    return res


def _host_only_object(src: str, obj: str) -> None:
    # host side only, sanitizers on the host side (each -fsanitize after -Xarch_host)
    cmd = [fvbuild.hipcc(), "--offload-arch=gfx950", "--offload-host-only", "-O1", "-g", "-fno-omit-frame-pointer",
           "-std=c++17", "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", '-DFV_BUILD_ID="sanitize"',
           "-I", fvbuild.INCLUDE, "-I", fvbuild.CSRC, "-c", src, "-o", obj]
    _run(cmd)


@pytest.fixture(scope="module")
def abi_driver(tmp_path_factory):
    if not (os.path.exists(CLANG) and shutil.which(fvbuild.hipcc())):
        pytest.skip("ROCm's clang / hipcc not available")
    d = tmp_path_factory.mktemp("sanitize")
    srcs = [os.path.join(fvbuild.CSRC, s) for s in fvbuild.SOURCES]
    objs = [str(d / (os.path.splitext(os.path.basename(s))[0] + ".o")) for s in srcs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        for f in [pool.submit(_host_only_object, s, o) for s, o in zip(srcs, objs)]:
            f.result()
    # the host objects name their (absent) device images; give each a placeholder
    stubs = []
    for o in objs:
        for line in _run(["nm", "-u", o]).stdout.splitlines():
            name = line.split()[-1]
            if name.startswith("__hip_fatbin"):
                stubs.append(name)
    stub_c = d / "fatbin_stubs.c"
    stub_c.write_text("".join(f"char {n}[16];\n" for n in sorted(set(stubs))))
    sflags = ["-fsanitize=" + ",".join(SAN), "-fno-sanitize-recover=undefined", "-g", "-O1", "-fno-omit-frame-pointer"]
    _run([CLANG_C, *sflags, "-c", str(stub_c), "-o", str(d / "fatbin_stubs.o")])
    _run([CLANG, *sflags, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c",
          os.path.join(HERE, "fake_hip.cpp"), "-o", str(d / "fake_hip.o")])
    _run([CLANG, *sflags, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", fvbuild.INCLUDE, "-c",
          os.path.join(HERE, "abi_driver.cpp"), "-o", str(d / "abi_driver.o")])
    exe = str(d / "abi_driver")
    _run([CLANG, *sflags, *objs, str(d / "fake_hip.o"), str(d / "abi_driver.o"), str(d / "fatbin_stubs.o"),
          "-lpthread", "-o", exe])
    return exe


def test_library_host_code_under_sanitizers(abi_driver):
    res = subprocess.run([abi_driver], capture_output=True, text=True, env={**os.environ, **ENV}, timeout=600)
    assert res.returncode == 0, f"exit {res.returncode}\n{res.stdout[-3000:]}\n{res.stderr[-12000:]}"
    assert "ok:" in res.stdout, res.stdout[-2000:]


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          os.path.join(ROOT, "oracle", "fv_oracle.c"), os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe])
    res = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, **ENV, "OMP_NUM_THREADS": "4"},
                         timeout=600)
    assert res.returncode == 0, f"exit {res.returncode}\n{res.stdout[-3000:]}\n{res.stderr[-12000:]}"
    assert "ok:" in res.stdout
