"""Build libx2c.so (gfx950) in-tree with hipcc.

Usage:  python -m paper_1303_4446_amd.builder   (or call build())
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libx2c.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["k_prep.hip", "k_gemm.hip", "k_large.hip", "k_tridiag.hip", "k_matvec.hip", "k_spectrum.hip", "k_lu.hip", "k_kramers.hip", "k_ozaki.hip", "k_ozaki_i8.hip", "k_dlu.hip", "k_fw.hip", "x2c_dkh_plan.cpp", "x2c_api.cpp"]

ARCH = os.environ.get("X2C_OFFLOAD_ARCH", "gfx950")
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, build_dir: str = BUILD_DIR, extra=()) -> str:
    os.makedirs(build_dir, exist_ok=True)
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIP_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
           "-x", "hip", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = LIB, build_dir: str = BUILD_DIR, extra=()) -> str:
    """Compile every HIP source for gfx950 and link libx2c.so (always rebuilds).
    `out`, `build_dir` and `extra` (more hipcc flags for every step) serve
    instrumented builds such as the host sanitizer test."""
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, tuple(extra)), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", *extra, f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if not extra:
        cmd.insert(3, "-Wl,--no-undefined")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
