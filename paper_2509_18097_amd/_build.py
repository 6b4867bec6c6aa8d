"""Builds libpdg.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_2509_18097_amd._build

Every HIP translation unit is compiled with hipcc for gfx950 only, with the
packed-FP32 instructions disabled, then linked into
``paper_2509_18097_amd/libpdg.so``.  Objects go to ``_build/`` at the
repository root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpdg.so")
ARCH = "gfx950"

SOURCES = ["sort.hip", "warp.hip", "chamfer.hip", "chamfer_screen.hip", "precond.hip",
           "dct.hip", "optim.hip", "keyframe.hip", "mesh.hip", "prune.hip", "api.hip"]

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC,
    # packed FP32 instructions have given silently wrong results on this
    # hardware generation: keep hipcc from forming them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results straight into VGPRs (no v_accvgpr_read copies); the
    # kernels consume every MFMA result with VALU instructions
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
]
# Per-file additions.  The nearest-neighbour screen takes finite coordinates
# only, so its minima need no NaN-quieting instruction per matrix-core
# result.
FILE_FLAGS = {"chamfer_screen.hip": ["-fno-honor-nans"]}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (need ROCm with gfx950 support)")


def _compile(src: str, hipcc: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc, *FLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if warn and os.environ.get("PDG_BUILD_VERBOSE"):
        print(warn, file=sys.stderr)
    return obj


def stale(lib: str = LIB) -> bool:
    """True when ``lib`` is missing or older than a HIP source, a header or
    this build script."""
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + \
        [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)] + [os.path.abspath(__file__)]
    return any(os.path.getmtime(d) > t for d in deps if os.path.isfile(d))


def build(jobs: int | None = None) -> str:
    """Compile every source and link libpdg.so; returns the library path."""
    hipcc = _hipcc()
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
