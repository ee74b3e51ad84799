"""Builds liblsgcpd.so (all HIP sources, gfx950) next to this file.

Usage: python -m paper_2103_15039_amd.build   (or build() from Python)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblsgcpd.so")
SOURCES = ["api.hip", "estep.hip", "mstep.hip", "knn_pca.hip", "order.hip", "confidence.hip",
           "proposal.hip"]
ARCH = os.environ.get("LSGCPD_ARCH", "gfx950")


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def command(out=LIB):
    return ([hipcc(), "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-shared",
             "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # keep MFMA accumulators in VGPRs (no AGPR round trips in the E-step loop)
             "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             # the first kernel arguments arrive in SGPRs at dispatch (no kernarg load
             # before a block's first dependent load; code for dispatchers without
             # preloading loads them itself)
             "-mllvm", "-amdgpu-kernarg-preload-count=16",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
            + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out])


def build(verbose=False):
    """Compiles every HIP source into liblsgcpd.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{errs}")
    if verbose and errs.strip():
        print(errs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
