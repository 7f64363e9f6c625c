"""Build libgleanvec.so (gfx950) in-tree with hipcc.

Usage: python paper_2410_22347_amd/build.py [--jobs N]
Each source is compiled to an object in ``_build/`` (parallel), then linked
into ``paper_2410_22347_amd/libgleanvec.so``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgleanvec.so")
ARCH = os.environ.get("GV_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # matrix-core results in ordinary VGPRs: the filters read them with
             # vector ALU ops, and accumulation-register copies would otherwise
             # force waits on the tile loads in flight
             "-mllvm", "-amdgpu-mfma-vgpr-form",
             "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-march=x86-64-v3"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _newest_dependency() -> float:
    """Latest modification time among the headers every source may include."""
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    heads.append(os.path.join(ROOT, "include", "gleanvec.h"))
    return max(os.path.getmtime(h) for h in heads)


def compile_one(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, src + ".o")
    path = os.path.join(CSRC, src)
    if incremental and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(os.path.getmtime(path), _newest_dependency()):
            return obj
    if src.endswith(".hip"):
        cmd = [hipcc(), *HIP_FLAGS, "-c", path, "-o", obj]
    else:
        cmd = ["g++", *CXX_FLAGS, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental: only those older than their object
    or than a header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = sources()
    jobs = jobs or min(8, os.cpu_count() or 4)
    # the scan instantiations are the slowest units: start them first
    order = sorted(hip, key=lambda f: not f.startswith("scan_")) + cpp
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: compile_one(f, incremental), order))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true", help="recompile only sources changed since their object")
    a = ap.parse_args()
    build(a.jobs, verbose=True, incremental=a.incremental)


if __name__ == "__main__":
    sys.exit(main())
