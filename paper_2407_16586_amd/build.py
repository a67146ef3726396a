"""Build libtdgrad.so (HIP, gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtdgrad.so")
TABLE = os.path.join(CSRC, "rys_table.inc")
GEN = os.path.join(CSRC, "gen_rys_table.py")
SOURCES = [os.path.join(CSRC, "tdgrad.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("tdg_device.hpp", "deriv_kernel.hpp")]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def table(force: bool = False) -> str:
    if force or not os.path.exists(TABLE) or os.path.getmtime(TABLE) < os.path.getmtime(GEN):
        subprocess.check_call([sys.executable, GEN, TABLE])
    return TABLE


def build(extra_flags: list[str] | None = None, verbose: bool = False) -> str:
    table()
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *(extra_flags or []), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(sys.argv[1:], verbose=True)
