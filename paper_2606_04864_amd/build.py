"""Build libamsp.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python paper_2606_04864_amd/build.py   (or call build()).
Object files go to _build/ at the repository root (git-ignored); the shared
library lands next to this file, where the Python binding loads it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libamsp.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I" + CSRC,
          "-I" + os.path.join(ROOT, "include"),
          # no packed-FP32 instructions anywhere in the device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]

SOURCES = ["k_krylov.hip", "k_local.hip", "k_apply.hip", "k_eigen.hip", "k_coarse.hip", "k_multi.hip",
           "k_tree.hip", "k_batch.hip", "amsp_tree.cpp",
           "amsp_plan.cpp",
           "amsp_host.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-6000:])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


def build_plan_check(out: str | None = None) -> str:
    """The host-only planner check program (csrc/plan_check.cpp) with
    AddressSanitizer and UndefinedBehaviorSanitizer: g++ on host code only,
    linked against the HIP runtime for its host API (page-locked blocks)."""
    out = out or os.path.join(BUILD, "plan_check")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    rocm = os.path.dirname(os.path.dirname(HIPCC))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(rocm, "include"), "-I" + CSRC,
           os.path.join(CSRC, "amsp_plan.cpp"), os.path.join(CSRC, "amsp_tree.cpp"),
           os.path.join(CSRC, "tree_check.cpp"), os.path.join(CSRC, "plan_check.cpp"),
           "-o", out, "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("plan_check build failed:\n" + r.stderr[-6000:])
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
