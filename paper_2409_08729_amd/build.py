"""Build liblbessel.so (HIP, gfx950) in-tree.

    python -m paper_2409_08729_amd.build

Generates csrc/lbessel_tables.h from exact rationals, then compiles
csrc/lbessel_kernels.hip (the kernels and their C-ABI) and
csrc/lbessel_serve.cpp (the serving runtime) with hipcc into
paper_2409_08729_amd/liblbessel.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbessel.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # exact control of rounding: every fused multiply-add is written as fma()
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep constant materialisation next to its use: hoisting the device
    # library's polynomial constants out of the grouped kernel's evaluation
    # loop costs ~140 VGPRs and two thirds of the occupancy
    "-mllvm", "-disable-machine-licm",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(out: str = LIB, extra: list[str] | None = None) -> str:
    sys.path.insert(0, HERE)
    try:
        import gen_tables
    finally:
        sys.path.pop(0)
    gen_tables.write_header()
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *(extra or []),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "lbessel_kernels.hip"),
           os.path.join(CSRC, "lbessel_serve.cpp"), "-lpthread", "-o", tmp]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed building liblbessel.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
