"""Build libigfilter.so for gfx950 in-tree with hipcc.

Every HIP source is compiled with -ffp-contract=off (multiply-adds only where
the source writes fmaf) and with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libigfilter.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC, "-Wno-unused-result"]


def _units():
    units = [("api", "api.cpp", ["-x", "hip"]), ("plan", "plan.cpp", []), ("reduce", "reduce.hip", []), ("batch", "batch.hip", []),
             ("quality", "quality.hip", []), ("sweep", "sweep.cpp", ["-x", "hip"]),
             ("smooth", "smooth.hip", []), ("wavelet", "wavelet.hip", []),
             ("noalloc", "noalloc.hip", [])]
    for c in range(3):
        for d in range(3):
            units.append((f"stencil_c{c}_d{d}", "stencil_inst.hip", [f"-DIG_COND={c}", f"-DIG_DTYPE={d}"]))
    extra = os.path.join(CSRC, "surrogate.hip")
    if os.path.exists(extra):
        units.append(("surrogate", "surrogate.hip", []))
    return units


def _compile(unit):
    name, src, flags = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{' '.join(cmd)}\n{r.stderr[-6000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile all units and link libigfilter.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, min(16, os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
