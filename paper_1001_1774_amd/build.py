"""Build the HIP library libtvcs.so for gfx950 in-tree with hipcc.

Run ``python -m paper_1001_1774_amd.build`` (or ``__graft_entry__.build()``).
Every source is compiled to an object in parallel (``_build/`` next to this file),
then the objects are linked into one shared library.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtvcs.so")
OBJDIR = os.path.join(PKG, "_build")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def flags(defines=(), extra=()):
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            *[f"-D{d}" for d in defines], *extra,
            "-Wall", "-Wno-unused-function", "-Wno-unused-result",
            # no packed-FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # MFMA accumulators in ordinary VGPRs: no AGPR copies in the product
            # loops, and fewer registers per wave
            "-mllvm", "-amdgpu-mfma-vgpr-form=1",
            f"-I{INCLUDE}", f"-I{CSRC}"]


def command(out: str = LIB, defines=(), extra=()):
    """One hipcc line that compiles and links every source (for reference)."""
    return [hipcc(), *flags(defines, extra), "-shared", *sources(), "-o", out]


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def build(verbose: bool = True, out: str = LIB, defines=(), extra=()) -> str:
    """Compile every source into one shared library (`defines`: extra -D tuning knobs,
    `extra`: extra compiler flags)."""
    tag = "_".join(d.replace("=", "-") for d in defines) or "default"
    objdir = os.path.join(OBJDIR, tag)
    os.makedirs(objdir, exist_ok=True)
    fl = flags(defines, extra)
    jobs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        jobs.append((src, obj, [hipcc(), *fl, "-c", src, "-o", obj]))
    if verbose:
        print(" ".join(jobs[0][2][:-4]) + " -c <each source>", flush=True)

    def run(job):
        src, obj, cmd = job
        r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True)
        err = "\n".join(l for l in (r.stderr or "").splitlines()
                        if "packed-fp32-ops" not in l)
        return src, r.returncode, err

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(run, jobs))
    failed = False
    for src, rc, err in results:
        if err.strip():
            print(f"--- {os.path.basename(src)}\n{err}", flush=True)
        failed |= rc != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = out + ".tmp"
    subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC",
                    *[obj for _, obj, _ in jobs], "-o", tmp], check=True, cwd=ROOT)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
