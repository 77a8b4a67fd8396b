"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code (CPU only).

- The oracle's C sources with ``tests/native/oracle_check.c``, which drives every oracle entry
  point on small boxes (general masks, thermal fluid and beads, MD substeps, excluded volume,
  the reverse pass, shell relaxation, error returns).
- The library's host-only planners (``paper_1604_01829_amd/csrc/lbrb_plan.cpp``: mask
  compression, node tiles, moving-wall links, bead order, excluded-volume site grids) with
  ``tests/native/plan_check.cpp``, which checks each against a brute-force definition.

Both are built with gcc/g++ (host code only: the planners include the HIP headers for their
types and make no HIP call), any sanitizer report aborts the program, and leaks are reported.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ORACLE_SOURCES = ["orc_lattice.c", "orc_philox.c", "orc_lbrb.c", "orc_adjoint.c", "orc_relax.c"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for bad in ("runtime error", "AddressSanitizer", "LeakSanitizer"):
        assert bad not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    cmd = (["gcc", "-std=c99", "-Wall", "-Wextra", "-Wno-unknown-pragmas", "-Werror"] + SAN +
           [os.path.join(ROOT, "oracle", s) for s in ORACLE_SOURCES] +
           [os.path.join(ROOT, "tests", "native", "oracle_check.c"), "-lm", "-o", exe])
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    assert "oracle_check: ok" in _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_host_planners_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = (["g++", "-std=c++17", "-Wall", "-Wextra", "-Wno-unknown-pragmas",
            "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + SAN +
           [os.path.join(ROOT, "tests", "native", "plan_check.cpp"),
            os.path.join(ROOT, "paper_1604_01829_amd", "csrc", "lbrb_plan.cpp"), "-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "orders and site grids ok" in _run(exe)
