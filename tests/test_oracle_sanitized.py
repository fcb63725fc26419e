"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU:

* the oracle: tests/sanitize/oracle_driver.c calls every oracle entry point
  on edge and random inputs (gcc, with OpenMP);
* the library's host-side arithmetic: tests/sanitize/host_driver.cpp runs the
  host build of the exact reductions, seeding, skip-ahead and the 3^40 step
  against the oracle (ROCm's clang as a plain host compiler, no GPU code).

Any sanitizer report or failed consistency check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")
CLANG = "/opt/rocm/llvm/bin/clang"


def _run(exe, marker):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert marker in r.stdout


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _build(["gcc", "-std=c11", "-fopenmp", "-fno-fast-math"] + SAN +
           ["-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "nn_oracle.c"),
            os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe])
    _run(exe, "oracle driver ok")


@pytest.mark.skipif(not os.path.exists(CLANG + "++"), reason="ROCm clang not available")
def test_host_arithmetic_under_sanitizers(tmp_path):
    obj = str(tmp_path / "nn_oracle.o")
    exe = str(tmp_path / "host_driver")
    _build([CLANG, "-std=c11", "-Wno-unknown-pragmas"] + SAN +
           ["-I", os.path.join(ROOT, "oracle"), "-c",
            os.path.join(ROOT, "oracle", "nn_oracle.c"), "-o", obj])
    _build([CLANG + "++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + SAN +
           ["-I", os.path.join(ROOT, "include"),
            "-I", os.path.join(ROOT, "paper_1206_1187_amd", "csrc"),
            "-I", os.path.join(ROOT, "oracle"),
            os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), obj, "-o", exe])
    _run(exe, "host driver ok")
