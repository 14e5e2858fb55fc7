"""Address, undefined-behaviour and leak sanitizer builds of the host-side
code, run on the CPU:

* the oracle (oracle.c) built with gcc -fsanitize=address,undefined: every
  oracle test module run against it, and a C driver of all its entry points
  (tests/pins/oracle_driver.c) built with the leak checker as well;
* the library's host code (fpt_host.cpp: descriptor validation, table build,
  scratch reservation, error paths) built with hipcc, the sanitizers on the
  host side only, linked with the ordinary kernels: the ABI tests and the
  table builds of every workload run against it.

The Python runs preload the sanitizer runtime and turn its leak checker off
(the interpreter keeps memory to the end by design); any error aborts the
child process and fails the test.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GCC_ASAN = "/usr/lib/gcc/x86_64-linux-gnu/11/libasan.so"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def _pytest(files, preload, **extra):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV, **extra)
    return _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                 "-m", "not gpu"] + files, env=env)


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    return str(tmp_path_factory.mktemp("san"))


@pytest.mark.skipif(not os.path.exists(GCC_ASAN), reason="gcc's address sanitizer runtime is missing")
def test_oracle_under_asan_ubsan(tmp):
    lib = os.path.join(tmp, "liboracle_san.so")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "oracle/oracle.c", "-lm",
          "-o", lib])
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    r = _pytest(files, GCC_ASAN, FPT_ORACLE_LIBRARY=lib)
    assert " passed" in r.stdout


@pytest.mark.skipif(not os.path.exists(GCC_ASAN), reason="gcc's address sanitizer runtime is missing")
def test_oracle_driver_under_asan_ubsan_lsan(tmp):
    exe = os.path.join(tmp, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined,leak",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-Ioracle",
          "tests/pins/oracle_driver.c", "oracle/oracle.c", "-lm", "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                             UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))
    assert r.stdout.strip() == "ok"


def _clang_asan():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return hits[0] if hits else None


@pytest.mark.skipif(not (os.path.exists(HIPCC) and _clang_asan()), reason="hipcc or its sanitizer runtime is missing")
def test_host_library_under_asan_ubsan(tmp):
    kernels = os.path.join(ROOT, "paper_1706_03024_amd", "_build", "fpt_kernels.o")
    if not os.path.exists(kernels):
        from paper_1706_03024_amd import build as b
        b.build()
    host = os.path.join(tmp, "fpt_host_san.o")
    lib = os.path.join(tmp, "libfpt_san.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops"] + san + ["-Iinclude", "-Ipaper_1706_03024_amd/csrc", "-c",
                                                  "paper_1706_03024_amd/csrc/fpt_host.cpp", "-o", host])
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + san[:4] + [kernels, host, "-o", lib])
    r = _pytest(["tests/test_abi.py", "tests/test_host_tables.py"], _clang_asan(), FPT_LIBRARY=lib)
    assert " passed" in r.stdout
