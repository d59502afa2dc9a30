"""Host logic of the batch's grouped launches: the work-group orders
(`csrc/wg_order.h`) keep every (product, tile) entry exactly once, keep the
tiles each order promises on one XCD, and fit the table capacity the library
allocates. The header is compiled with the system C++ compiler; no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_09244_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_work_group_orders(tmp_path):
    exe = tmp_path / "wg_order_check"
    src = os.path.join(ROOT, "tests", "wg_order_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
