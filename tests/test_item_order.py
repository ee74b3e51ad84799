"""The pair kernel's block -> work-item order (estep.hip, item_order) is a
permutation of a problem's items that gives each XCD a contiguous run of
them and, when every source group has the same number of items, runs each
XCD's groups item by item: a host build of the function, checked on sizes
from one item to thousands.  The order changes no result (every item is
run exactly once and the partial sums are combined by item number)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_item_order_is_a_permutation_with_xcd_runs():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "item_order_check")
        subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-I", os.path.join(ROOT, "paper_2103_15039_amd", "csrc"),
                        "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "item_order_check.hip"), "-o", exe],
                       check=True, capture_output=True, timeout=600)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
