"""The C-ABI host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Compiles the host code (``csrc/ssfm.cpp``) with the sanitizers on its host
side only (``-Xarch_host``; the device code is not instrumented), links it
with the kernel objects of the in-tree build and the driver
``tests/sanitize/host_abi.cpp``, and runs the driver on the CPU: workspace
sizing, the checkpoint planner, plan-variant counts and every argument
check that returns before a device call.  Any sanitizer report fails the
test.
"""
import os
import shutil
import subprocess

import pytest

from paper_2306_15678_amd.build import UNITS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2306_15678_amd")
BUILD = os.path.join(PKG, "_build")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
       "-fno-omit-frame-pointer"]


def test_host_abi_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    objs = [os.path.join(BUILD, u + ".o") for u in UNITS]
    if not os.path.exists(hipcc) or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc and the kernel objects of the in-tree build")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    host_o = str(tmp_path / "ssfm_san.o")
    drv_o = str(tmp_path / "host_abi.o")
    exe = str(tmp_path / "host_abi")
    steps = [
        [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++20", *inc, *SAN, "-c",
         os.path.join(PKG, "csrc", "ssfm.cpp"), "-o", host_o],
        [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++20", *inc, *SAN, "-c",
         os.path.join(ROOT, "tests", "sanitize", "host_abi.cpp"), "-o", drv_o],
        [hipcc, "--offload-arch=gfx950", *SAN, drv_o, host_o, *objs, "-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout + r.stderr
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert r.returncode == 0 and "all checks passed" in out, out
