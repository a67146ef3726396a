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
MAIN = os.path.join(CSRC, "tdgrad.hip")
CLASS_SRC = os.path.join(CSRC, "class_kernels.hip")
FOCK_SRC = os.path.join(CSRC, "fock_kernels.hip")
NUM_CLASSES = 21

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


# sources each object depends on (for incremental builds)
_DEV = ["tdg_device.hpp", "rys_table.inc"]
_DEPS = {
    "tdgrad": ["tdgrad.hip", "class_launch.hpp", "deriv_kernel.hpp", "fock_kernel.hpp", "fock_launch.hpp", "mlp.hpp",
               "../../include/tdgrad.h"] + _DEV,
    "mlp": ["mlp.hip", "mlp.hpp", "../../include/tdgrad.h"],
    "zvector": ["zvector.hip", "../../include/tdgrad.h"],
    "class": ["class_kernels.hip", "class_launch.hpp", "deriv_kernel.hpp", "deriv_wave.hpp"] + _DEV,
    "fock": ["fock_kernels.hip", "fock_launch.hpp", "fock_kernel.hpp", "deriv_kernel.hpp"] + _DEV,
}


def build(extra_flags: list[str] | None = None, verbose: bool = False, jobs: int | None = None,
          incremental: bool = False) -> str:
    """Compile the host runtime and the 21 per-class kernel units in parallel, then link.
    incremental=True keeps the objects in _build/ and recompiles only those whose
    sources changed since (same flags assumed)."""
    import concurrent.futures as cf
    import tempfile

    table()
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"] + list(extra_flags or [])
    tmp_ctx = tempfile.TemporaryDirectory(prefix="tdgrad_build_")
    with tmp_ctx as tmpd:
        odir = os.path.join(os.path.dirname(CSRC), "_build") if incremental else tmpd
        os.makedirs(odir, exist_ok=True)
        jobs_ = [(MAIN, os.path.join(odir, "tdgrad.o"), [], "tdgrad"),
                 (os.path.join(CSRC, "mlp.hip"), os.path.join(odir, "mlp.o"), [], "mlp"),
                 (os.path.join(CSRC, "zvector.hip"), os.path.join(odir, "zvector.o"), [], "zvector")]
        for c in range(NUM_CLASSES):
            jobs_.append((CLASS_SRC, os.path.join(odir, f"class_{c}.o"), [f"-DTDG_CLASS={c}"], "class"))
        for c in range(NUM_CLASSES):
            jobs_.append((FOCK_SRC, os.path.join(odir, f"fock_{c}.o"), [f"-DTDG_CLASS={c}"], "fock"))

        def stale(obj, kind):
            if not incremental or not os.path.exists(obj):
                return True
            t = os.path.getmtime(obj)
            return any(os.path.getmtime(os.path.join(CSRC, d)) > t for d in _DEPS[kind])

        def compile_one(job):
            src, obj, defs, kind = job
            if not stale(obj, kind):
                return 0, "", obj
            cmd = [hipcc, *flags, *defs, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
            return r.returncode, r.stdout + r.stderr, obj

        n = jobs or min(len(jobs_), max(1, min(16, os.cpu_count() or 1)))
        with cf.ThreadPoolExecutor(n) as ex:
            results = list(ex.map(compile_one, jobs_))
        for rc, out, obj in results:
            if verbose or rc:
                sys.stderr.write(out)
            if rc:
                raise RuntimeError(f"compilation of {obj} failed")
        tmp = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [r[2] for r in results]
        subprocess.check_call(cmd, cwd=CSRC)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(sys.argv[1:], verbose=True)
