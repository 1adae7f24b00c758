"""Build the HIP library for gfx950 with hipcc (in-tree).

``libppml.so``       -- the product library (FMA contraction on, divisions by
                        constants and cell sizes replaced by multiplications).
``libppml_exact.so`` -- the same source with PPML_EXACT: no FMA contraction and
                        every division where the scheme's formulas divide, for
                        operation-by-operation FP64 comparisons in the tests.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SRC = os.path.join(CSRC, "ppml_api.hip")
LIB = os.path.join(CSRC, "libppml.so")
LIB_EXACT = os.path.join(CSRC, "libppml_exact.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BASE_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed FP32 instructions (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _command(out: str, exact: bool) -> list[str]:
    flags = list(BASE_FLAGS)
    if exact:
        flags += ["-DPPML_EXACT=1", "-ffp-contract=off"]
    else:
        # FP32 division and square root at hardware rate (1 ulp) and FP32
        # subnormals flushed to zero, which drops the operand scaling around
        # v_rcp_f32 / v_sqrt_f32 (no state value of a physical run comes near
        # 1e-38); FP64 keeps correctly rounded division, square root and
        # subnormals
        flags += ["-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero"]
    # rocBLAS runs the GEMMs of the self-gravity sine transforms
    return [HIPCC, *flags, SRC, "-o", out + ".tmp", "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]


def build_one(out: str, exact: bool) -> str:
    r = subprocess.run(_command(out, exact), capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {out}")
    os.replace(out + ".tmp", out)
    return out


def build() -> list[str]:
    """Both libraries, compiled side by side."""
    jobs = [(out, subprocess.Popen(_command(out, exact), stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
            for out, exact in ((LIB, False), (LIB_EXACT, True))]
    failed = []
    for out, proc in jobs:
        log, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(log)
            failed.append(out)
    if failed:
        raise RuntimeError(f"hipcc failed for {', '.join(failed)}")
    for out, _ in jobs:
        os.replace(out + ".tmp", out)
    return [out for out, _ in jobs]


if __name__ == "__main__":
    for p in build():
        print(p)
