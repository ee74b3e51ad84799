"""The key that orders both clouds (order.hip) is a 3-D Hilbert curve: a
host build of the key function, checked for its start and end, for filling
the 64^3 corner cube with the first 2^18 keys exactly once, and for face
adjacency of consecutive keys at a million random cells.  The order changes
no result of the library beyond rounding; it decides how tight the boxes of
consecutive points are, and so how many pairs the E step can skip."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_curve_key_is_a_hilbert_curve():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "curve_order_check")
        subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
                        "-I", os.path.join(ROOT, "paper_2103_15039_amd", "csrc"),
                        "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "curve_order_check.hip"), "-o", exe],
                       check=True, capture_output=True, timeout=600)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
