"""Build libssfm.so (HIP kernels for gfx950 + the C-ABI host code) in-tree.

    python -m paper_2306_15678_amd.build

The pass kernels are compiled in five units (row / column x complex64 /
complex128, and the half-exchange column passes) in parallel with the pointwise kernels and the host code, then
linked with hipcc.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libssfm.so")
ARCH = os.environ.get("SSFM_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++20", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# packed FP32 instructions are disabled for all device code
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# device units (csrc/<unit>.hip), compiled in parallel
UNITS = ["kernels", "diagnostics", "pass_row_f32", "pass_row_f64", "pass_col_f32",
         "pass_col_f64", "pass_col_hx_f32"]


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm toolchain required to build)")
    return exe


def _sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith((".hip", ".hpp", ".cpp", ".h"))] + \
        [os.path.join(ROOT, "include", "ssfm.h")]


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile and link; returns the library path."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in _sources())
        if os.path.getmtime(LIB) >= newest:
            return LIB
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    units = UNITS
    jobs = [[hipcc, f"--offload-arch={ARCH}", *COMMON, *DEVICE, "-c",
             os.path.join(CSRC, u + ".hip"), "-o", os.path.join(BUILD, u + ".o")] for u in units]
    jobs.append([hipcc, f"--offload-arch={ARCH}", *COMMON, "-Wall", "-c",
                 os.path.join(CSRC, "ssfm.cpp"), "-o", os.path.join(BUILD, "ssfm.o")])
    objs = [os.path.join(BUILD, u + ".o") for u in units] + [os.path.join(BUILD, "ssfm.o")]
    t0 = time.time()
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
             for j in jobs]
    failed = []
    for j, p in zip(jobs, procs):
        out, _ = p.communicate()
        if verbose and out:
            sys.stdout.write(out)
        if p.returncode != 0:
            failed.append((j, out))
    if failed:
        msg = "\n".join(" ".join(j) + "\n" + out for j, out in failed)
        raise RuntimeError("libssfm build failed:\n" + msg)
    tmp = LIB + ".tmp"
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("libssfm link failed:\n" + " ".join(link) + "\n" + r.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s")
    return LIB


if __name__ == "__main__":
    build(verbose=True, force=True)
