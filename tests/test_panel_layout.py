"""Host check of the panel-packed layout builder and of the kernel's run-sum order.

`panel_layout_check.cpp` is compiled with the library's host layout builder (lp_layout.cpp,
no GPU code) and run: on 300 random matrices it walks every unit the way the panel SpMV kernel
does (64-entry chunks, pieces at row-id drops, runs added in order by their first entry) and
requires every row sum to equal the plain CSR-order sum bit for bit; it also checks the packed
entries, the row cap and that the unit count never exceeds its target when the cap allows.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2604_23951_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_panel_layout_and_run_sum_order(tmp_path):
    exe = str(tmp_path / "panel_layout_check")
    # the host sanitizer run (test_host_sanitizers.py) substitutes an instrumented compiler line
    cxx = os.environ.get("HOST_CXX", "g++").split()
    cmd = [*cxx, "-O2", "-std=c++17", "-Wall", "-I", CSRC, "-o", exe,
           os.path.join(HERE, "panel_layout_check.cpp"), os.path.join(CSRC, "lp_layout.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    ok, trials, chunks, multi = r.stdout.split()
    assert ok == "ok" and int(trials) == 300
    assert int(multi) > 0  # chunks that cross a panel segment boundary were exercised
