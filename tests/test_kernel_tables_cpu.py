"""CPU check of the class kernels' per-lane integral tables (csrc/deriv_kernel.hpp compiled as
host code through tests/cpu/shim): for every one of the 21 classes, every table entry that
the kernels read -- the vertical-recursion + transfer tables with their raised and lowered
entries, the direct four-centre base tables and their derivative tables -- is written by
the recursion first.  A read of an unwritten entry would take what the lane's private
memory held before (scratch, when a kernel spills) and make a result depend on earlier
launches.  A table bound shortened by one in the transfer step fails it (159 reads)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_every_read_table_entry_is_written(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "table_coverage")
    subprocess.check_call([cxx, "-std=c++17", "-O1", "-Wno-unknown-pragmas", "-I", os.path.join(HERE, "cpu", "shim"),
                           "-o", exe, os.path.join(HERE, "cpu", "table_coverage.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.startswith("OK 63"), out.stdout
