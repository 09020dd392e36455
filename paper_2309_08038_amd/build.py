"""Build librosar.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2309_08038_amd.build [--jobs N] [--save-temps DIR]
Objects go to _build/ at the repository root; the library to paper_2309_08038_amd/librosar.so.
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
LIB = os.path.join(PKG, "librosar.so")
SOURCES = ["range_compress.hip", "sparse_filter.hip", "fastconv.hip", "adjoint_band.hip", "bp_full.hip", "bp_time_domain.hip", "cartesian.hip", "sas_design.hip", "delta_r.hip", "beampattern.hip", "backward.hip",
           "batch.hip", "api.cpp", "autotune_cache.cpp"]
ARCH = "gfx950"

# Packed FP32 instructions stay off: the compiler would otherwise form v_pk_fma_f32 and
# friends from ordinary float code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build librosar)")


def _compile(src: str, save_temps: str | None) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if save_temps:
        os.makedirs(save_temps, exist_ok=True)
        cmd += ["--save-temps"]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=save_temps or BUILD)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 8, save_temps: str | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, save_temps), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking librosar.so failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--save-temps", default=None, help="directory for device assembly (.s) files")
    a = ap.parse_args(argv)
    build(a.jobs, a.save_temps, verbose=True)


if __name__ == "__main__":
    sys.exit(main())
