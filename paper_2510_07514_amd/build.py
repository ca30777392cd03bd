"""Build libhjcd.so for gfx950 in-tree (``python -m paper_2510_07514_amd.build``).

Every HIP translation unit is compiled by hipcc for --offload-arch=gfx950 in
parallel (the per-seed solve kernel once per joint-count bucket), then linked
into ``paper_2510_07514_amd/libhjcd.so``.  Packed-FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhjcd.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ARCH = "gfx950"
NM_BUCKETS = (6, 7, 8, 12, 16, 20, 24, 32)  # 6 and 7: exact joint counts
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", CSRC, "-I", INCLUDE]


def _units():
    units = [("hjcd_kernels.o", "hjcd_kernels.hip", []),
             ("hjcd_api.o", "hjcd_api.cpp", ["-x", "hip"]),
             ("hjcd_server.o", "hjcd_server.cpp", ["-x", "hip"]),
             ("hjcd_plan.o", "hjcd_plan.cpp", ["-x", "hip"])]
    for nm in NM_BUCKETS:
        units.append((f"hjcd_solve_nm{nm}.o", "hjcd_solve_inst.hip", [f"-DHJCD_NM={nm}"]))
    return units


def _compile(unit, verbose, flags, build_dir):
    obj, src, extra = unit
    cmd = [HIPCC] + COMMON + flags + extra + ["-c", os.path.join(CSRC, src), "-o", os.path.join(build_dir, obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {extra}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None, flags=(), lib_path: str = LIB,
          build_dir: str = BUILD) -> str:
    """Compile every unit (extra hipcc `flags`, e.g. -DHJCD_WAVES_PER_EU=3) and
    link the library at `lib_path`; returns the library path."""
    os.makedirs(build_dir, exist_ok=True)
    units = _units()
    flags = list(flags)
    jobs = jobs or min(len(units), max(1, min(os.cpu_count() or 4, 8)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose, flags, build_dir), units))
    tmp = lib_path + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
          [os.path.join(build_dir, o) for o in objs] + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
