"""Build libnsrgs.so (HIP for gfx950) in the package directory.

Every translation unit keeps its device assembly (-save-temps), and the build
fails if any kernel runs vector work under a narrowed exec mask at a branch
join (see asmcheck.py).

Usage: python -m paper_2604_07372_amd.build  [--jobs N] [--verbose]
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

try:
    from . import asmcheck
except ImportError:          # run as a script
    import asmcheck

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libnsrgs.so")

SOURCES = (["batched_f64.hip", "batched_f32.hip", "batched_bf16.hip"]
           + [f"symmetric_{f}.hip" for f in ("split", "f64", "bf16", "f32")]
           + [f"stream_{f}_{part}.hip" for f in ("fp8", "split", "f64", "bf16", "f32") for part in ("m0c", "m0b", "m0a", "m1")]
           + ["stream.hip", "init.hip", "gen.hip", "runtime.hip", "batched.hip", "server.hip", "autotune.hip", "symmetric.hip", "bsr.hip", "noalloc.hip", "wide.hip", "stiefel.hip"])

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, "-save-temps=obj", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libnsrgs.so.  Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    device_asm = [os.path.join(BUILD, os.path.splitext(s)[0] + "-hip-amdgcn-amd-amdhsa-gfx950.s") for s in srcs]
    problems = asmcheck.check_files([p for p in device_asm if os.path.exists(p)])
    if problems:
        raise RuntimeError("generated code runs vector work under a narrowed exec mask:\n" + "\n".join(problems))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
