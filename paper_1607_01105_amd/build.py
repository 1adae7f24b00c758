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


def build_one(out: str, exact: bool) -> str:
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
    tmp = out + ".tmp"
    # rocBLAS runs the GEMMs of the self-gravity sine transforms
    cmd = [HIPCC, *flags, SRC, "-o", tmp, "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {out}")
    os.replace(tmp, out)
    return out


def build() -> list[str]:
    return [build_one(LIB, False), build_one(LIB_EXACT, True)]


if __name__ == "__main__":
    for p in build():
        print(p)
