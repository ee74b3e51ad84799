"""The C ABI without a GPU: the library loads, exports every function that
include/lsgcpd.h declares, the header compiles as C and C++, the struct
layouts match the Python binding, and opening a context fails cleanly when no
device is present."""
import ctypes as C
import os
import re
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsgcpd.h")

import paper_2103_15039_amd as L


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lsgcpd_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load_library()
    names = _declared()
    assert set(L.SYMBOLS) == set(names)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (lsgcpd_\w+)", out))
    assert exported == set(names)
    assert lib.lsgcpd_abi_version() == L.ABI_VERSION == 6
    assert lib.lsgcpd_status_string(3) == b"LSGCPD_E_NOMEM"


@pytest.mark.parametrize("cc,ext", [("gcc", "c"), ("g++", "cpp")])
def test_header_compiles_and_layout_matches(cc, ext):
    prog = r'''
#include <stddef.h>
#include <stdio.h>
#include "lsgcpd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lsgcpd_pose),
         sizeof(lsgcpd_estep_out), offsetof(lsgcpd_estep_out, stats),
         offsetof(lsgcpd_estep_out, newton_iters), sizeof(lsgcpd_params),
         offsetof(lsgcpd_params, tol), sizeof(lsgcpd_report), offsetof(lsgcpd_report, sigma2),
         sizeof(lsgcpd_profile), offsetof(lsgcpd_profile, evaluated_pairs),
         offsetof(lsgcpd_params, eta), offsetof(lsgcpd_report, w0),
         offsetof(lsgcpd_report, m_used));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, f"t.{ext}")
        exe = os.path.join(d, "t")
        open(src, "w").write(prog)
        subprocess.run([cc, "-std=c99" if ext == "c" else "-std=c++11", "-Wall", "-Werror",
                        "-I", os.path.dirname(HEADER), src, "-o", exe], check=True)
        got = list(map(int, subprocess.run([exe], capture_output=True, text=True).stdout.split()))
    want = [C.sizeof(L.Pose), C.sizeof(L.EstepOut), L.EstepOut.stats.offset,
            L.EstepOut.newton_iters.offset, C.sizeof(L.Params), L.Params.tol.offset,
            C.sizeof(L.Report), L.Report.sigma2.offset, C.sizeof(L.Profile),
            L.Profile.evaluated_pairs.offset, L.Params.eta.offset, L.Report.w0.offset,
            L.Report.m_used.offset]
    assert got == want


def test_params_default():
    p = L.default_params()
    assert (p.k, p.alpha_max, p.lambda_, p.w0, p.max_iter, p.newton_max) == (10, 30.0, 0.2, 0.1, 50, 20)
    assert (p.flags, p.eta, p.V, p.tol, p.sigma2_init) == (0, 0.0, 0.0, 0.0, 0.0)


def test_context_without_device_fails_cleanly():
    code = ("import ctypes as C, paper_2103_15039_amd as L; lib = L.load_library(); "
            "h = C.c_void_p(); print(lib.lsgcpd_ctx_create(0, C.byref(h)), "
            "lib.lsgcpd_ctx_create(-1, C.byref(h)))")
    env = dict(os.environ, HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    a, b = map(int, r.stdout.split())
    assert b == L.E_HIP
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    assert a == (L.OK if has_gpu else L.E_HIP)
