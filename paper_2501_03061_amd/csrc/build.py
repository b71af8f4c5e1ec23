"""Builds libpx.so (gfx950) from the sources in this directory.

    python -m paper_2501_03061_amd.csrc.build      # or build() from Python

Every .hip translation unit is compiled with hipcc for gfx950 only; the pair
pipeline is compiled once per grid size (-DPX_N=n) so the sizes build in
parallel.  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libpx.so")
BUILD_DIR = os.path.join(HERE, "_build")
SIZES = (16, 24, 32, 40, 48, 60, 64, 72, 80, 96)
# non-cubic grids (x, y, z): the wavefunction grids of the paper's 768- and
# 1536-atom cells
SHAPES = ((60, 60, 90), (60, 90, 120))
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", HERE,
          "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _units():
    units = []
    for n in SIZES:
        units.append(("exchange_inst.hip", f"exchange_n{n}.o", [f"-DPX_N={n}"]))
    for n0, n1, n2 in SHAPES:
        units.append(("exchange_shape.hip", f"exchange_s{n0}x{n1}x{n2}.o",
                      [f"-DPX_S0={n0}", f"-DPX_S1={n1}", f"-DPX_S2={n2}"]))
    for src in ("exchange_dispatch.cpp", "pair_transpose.hip", "misc_kernels.hip", "gemm_kernels.hip",
                "chol_kernels.hip", "eig_kernels.hip", "density_fine.hip", "px_api.cpp"):
        units.append((src, os.path.splitext(src)[0] + ".o", []))
    return units


def _compile(unit):
    src, obj, extra = unit
    cmd = [_hipcc(), "-x", "hip", "-c", os.path.join(HERE, src), "-o",
           os.path.join(BUILD_DIR, obj)] + COMMON + DEVICE + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stderr or "").splitlines()
                     if "packed-fp32-ops" not in l)
    return src, obj, r.returncode, msgs


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    units = _units()
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, units))
    failed = [r for r in results if r[2] != 0]
    for src, obj, rc, msgs in results:
        if msgs.strip() and (verbose or rc != 0):
            print(f"--- {src} -> {obj}\n{msgs}", file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(f"{s} ({o})" for s, o, _, _ in failed))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + \
          [os.path.join(BUILD_DIR, o) for _, o, _ in units]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
