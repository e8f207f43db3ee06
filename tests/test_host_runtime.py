"""The library's host code under AddressSanitizer and ThreadSanitizer (CPU only).

The HIP sources are compiled for the host side only, with the sanitizer on the
host pass, and linked against a stand-in runtime (tests/hostrt/hip_standin.cpp)
in place of the HIP runtime: kernels are no-ops, stream work is deferred to the
next synchronise (as HIP permits), device memory is sanitizer-tracked host
memory, and graph calls from several threads at once are flagged.  The driver
(tests/hostrt/served_driver.cpp) builds plain geometries and applies from the
main thread, then runs served mode with graph replay: sixteen client threads,
forty sessions, eight lanes; then the same with batching on two lanes, where
sessions of one kind share a lane and run in batched launches.

These runs catch a host buffer released while a queued copy may still read it
(the geometry set-up's reciprocal table once was), and graph calls that the
lanes do not serialise.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_20809_amd", "csrc")
HOSTRT = os.path.join(ROOT, "tests", "hostrt")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
CLANG = "/opt/rocm/llvm/bin/clang"
SOURCES = ["capi", "setup", "apply", "far_mfma", "far_stokes", "far_multi", "stokes", "server", "solve", "deriv", "targets", "stokes_dl", "tree"]

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)),
                                reason="needs the ROCm compilers")


def _run(cmd, cwd):
    res = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{res.stderr[-4000:]}")
    return res


def _build(san: str, out: str) -> str:
    """Compile the library's host code and the stand-in with -fsanitize=<san> on the host pass."""
    os.makedirs(out, exist_ok=True)
    san_flags = ["-Xarch_host", f"-fsanitize={san}"]
    common = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17"]

    def hip_obj(name):
        obj = os.path.join(out, name + ".o")
        _run([HIPCC, "--offload-arch=gfx950", "--offload-host-only", *common, "-fPIC", *san_flags, "-c",
              os.path.join(CSRC, name + ".hip"), "-o", obj], out)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(hip_obj, SOURCES))
    inc = ["-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")]
    standin = os.path.join(out, "standin.o")
    _run([CLANGXX, *common, *san_flags, "-D__HIP_PLATFORM_AMD__", *inc, "-Wno-unused-value", "-c",
          os.path.join(HOSTRT, "hip_standin.cpp"), "-o", standin], out)
    driver = os.path.join(out, "driver.o")
    _run([CLANGXX, *common, *san_flags, *inc, "-c", os.path.join(HOSTRT, "served_driver.cpp"), "-o", driver], out)
    # the host objects name each translation unit's device image; the stand-in
    # loads none, so empty definitions satisfy the references
    names = set()
    for o in objs:
        names.update(re.findall(r"__hip_fatbin_[0-9a-f]+", _run(["nm", "-u", o], out).stdout))
    stubs = os.path.join(out, "fatbin_stubs.c")
    with open(stubs, "w") as f:
        f.writelines(f"char {n}[16];\n" for n in sorted(names))
    _run([CLANG, "-c", stubs, "-o", stubs + ".o"], out)
    exe = os.path.join(out, "served_driver")
    _run([CLANGXX, f"-fsanitize={san}", *objs, standin, driver, stubs + ".o", "-o", exe, "-lpthread"], out)
    return exe


@pytest.mark.parametrize("san", ["address", "thread"])
def test_host_code_under_sanitizer(san, tmp_path):
    exe = _build(san, str(tmp_path))
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["TSAN_OPTIONS"] = "halt_on_error=0:exitcode=66"
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    log = res.stdout + res.stderr
    assert "ERROR: AddressSanitizer" not in log, log[-6000:]
    assert "WARNING: ThreadSanitizer" not in log, log[-6000:]
    assert "LeakSanitizer" not in log, log[-6000:]
    assert res.returncode == 0, log[-6000:]
    assert "served: admitted 40, applies 200, lanes 8, graphs 1\n" in log, log[-2000:]
    assert "served: admitted 40, applies 200, lanes 2, graphs 1, batched" in log, log[-2000:]
    assert "served tree: applies 6, tree sessions 2" in log, log[-2000:]
    assert "violations 0" in log, log[-2000:]
    shutil.rmtree(str(tmp_path), ignore_errors=True)
