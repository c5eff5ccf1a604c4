"""Build libemagpie.so for gfx950 with hipcc (in-tree, next to the Python binding).

Usage: python -m paper_2511_01793_amd.csrc.build   (or call build()).
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libemagpie.so")
SOURCES = ["kernels_m32.hip", "kernels_m64.hip", "kernels_m128.hip", "kernels_m256.hip", "kernels_peak.hip", "noalloc.hip",
           "kernels_common.hip", "api.hip"]

# Packed FP32 VALU forms are disabled on purpose: every FP32 operation is a
# scalar-lane IEEE operation.  hipcc's host pass does not know this feature
# and says so; that message is harmless.  Floating-point contraction is off so
# that every operation is rounded on its own: the same source arithmetic then
# gives the same bits in every kernel that inlines it (all launch strategies
# agree bitwise).  Up to six leading kernel arguments are preloaded into scalar
# registers at dispatch (the patch and finalize kernels put the pointers their
# first loads need there).
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-kernarg-preload-count=6",
    "-I" + os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; the HIP toolchain (ROCm) is required")
    return p


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc, *HIPFLAGS, "-c", os.path.join(HERE, s), "-o", o] for s, o in zip(SOURCES, objs)]
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for r in ex.map(_run, cmds):
            if verbose:
                sys.stdout.write(r.stdout + r.stderr)
    tmp = OUT + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
