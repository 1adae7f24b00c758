"""Sanitizer builds, on the CPU: the oracle and the host-side code of the
HIP library, each built with AddressSanitizer and UndefinedBehaviorSanitizer
(no recovery: the first finding aborts) and run by a driver under
tests/sanitize.  The oracle's driver steps every mode it has on small grids;
the library's driver exercises descriptor validation, sizing, the tile
tables, the NULL-handle checks and the HIP-error paths with no device.
Leak detection is on.  (GPU code is not instrumented: the sanitizers act on
host code only.)"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[0], r.returncode, (r.stdout + r.stderr)[-4000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(ROOT, "oracle", "ppml_oracle.c"), os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "0 failure(s)" in r.stdout


def test_host_library_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    exe = str(tmp_path / "host_san")
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    _run([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Wno-unused-command-line-argument",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
          os.path.join(ROOT, "paper_1607_01105_amd", "csrc", "ppml_api.hip"), os.path.join(SAN, "host_driver.cpp"),
          "-o", exe, "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"], timeout=900)
    # without a device the library's HIP calls fail and take their error
    # paths; on a machine with a GPU the driver stops at the first call that
    # expects that failure, so it is run with every device hidden
    env = dict(ENV, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    r = _run([exe], env=env, timeout=300)
    assert "0 failure(s)" in r.stdout
