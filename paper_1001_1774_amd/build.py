"""Build the HIP library libtvcs.so for gfx950 in-tree with hipcc.

Run ``python -m paper_1001_1774_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtvcs.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def command(out: str = LIB, defines=(), extra=()):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            *[f"-D{d}" for d in defines], *extra,
            "-Wall", "-Wno-unused-function", "-Wno-unused-result",
            # no packed-FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # MFMA accumulators in ordinary VGPRs: no AGPR copies in the product
            # loops, and fewer registers per wave
            "-mllvm", "-amdgpu-mfma-vgpr-form=1",
            f"-I{INCLUDE}", f"-I{CSRC}", *sources(), "-o", out]


def build(verbose: bool = True, out: str = LIB, defines=(), extra=()) -> str:
    """Compile every source into one shared library (`defines`: extra -D tuning knobs,
    `extra`: extra compiler flags)."""
    tmp = out + ".tmp"
    cmd = command(tmp, defines, extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=ROOT)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
