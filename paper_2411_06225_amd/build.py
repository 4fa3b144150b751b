"""Build librpr.so (HIP kernels for gfx950 + the C ABI) in-tree.

Each (right-hand side, precision) pair of the propagator and chain kernels is
its own translation unit, so the objects compile in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librpr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
         # no packed FP32 instructions in any kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]
KINDS = {0: "burgers", 1: "diffreact", 2: "bruss", 3: "swe", 4: "bruss3d"}
# the on-chip and tiled propagators serve the 1D and 2D systems; the generic
# one (any tableau) and the chain serve every system
UNIT_KINDS = {"propagate": (0, 1, 2, 3), "tiled": (0, 1, 2, 3), "chain": (0, 1, 2, 3, 4), "rkgen": (0, 1, 2, 3, 4)}
REALS = ("double", "float")


def _units():
    units = []
    for src, kinds in UNIT_KINDS.items():
        for k in kinds:
            kname = KINDS[k]
            for real in REALS:
                obj = os.path.join(BUILD, f"{src}_{kname}_{real}.o")
                units.append((os.path.join(CSRC, src + ".hip"), obj, [f"-DRPR_KIND={k}", f"-DRPR_REAL={real}"]))
    for src in ("randnet", "dispatch", "api", "autotune", "batch", "blocks", "stability"):
        units.append((os.path.join(CSRC, src + ".hip"), os.path.join(BUILD, src + ".o"), []))
    return units


def _compile(unit):
    src, obj, defs = unit
    cmd = [HIPCC] + FLAGS + defs + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-Wl,--version-script=" + os.path.join(CSRC, "exports.map")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
