"""Build libaco.so (all HIP sources, gfx950) in-tree with hipcc.

    python -m paper_1709_03187_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libaco.so")
SOURCES = ["candidates.hip", "construct.hip", "update.hip", "batch.hip", "mlp.hip", "two_opt.hip",
           "capi.hip"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off",                                      # no FMA contraction anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


STEP_PROFILE_OUT = os.path.join(PKG, "libaco_step_profile.so")


def build(verbose: bool = False, step_profile: bool = False) -> str:
    """Compile every source to an object, then link libaco.so (always rebuilds).
    step_profile: build libaco_step_profile.so instead, whose construction
    kernels also record per-ant clock counters (see step_profile.py)."""
    cc = hipcc()
    bdir = os.path.join(PKG, "_build_step_profile" if step_profile else "_build")
    out = STEP_PROFILE_OUT if step_profile else OUT
    extra = ["-DACO_STEP_PROFILE"] if step_profile else []
    os.makedirs(bdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [cc, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True, cwd=bdir)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        # the host pass does not know the packed-FP32 feature flag: harmless, drop it
        err = "\n".join(line for line in r.stderr.splitlines()
                        if line.strip() and "packed-fp32-ops' is not a recognized" not in line)
        if verbose and err:
            print(err, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + f".tmp{os.getpid()}"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=bdir)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, step_profile="--step-profile" in sys.argv[1:]))
