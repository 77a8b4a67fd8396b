"""Build the gfx950 shared library ``paper_1604_01829_amd/liblbrb.so`` with hipcc.

The library holds the HIP kernels and the C-ABI of ``include/lbrb.h``.  Packed FP32
instructions are disabled for the device code (-packed-fp32-ops); the host pass of hipcc
warns that it does not know that feature, which is harmless.  Multiply-adds are fused only
within one source expression (-ffp-contract=on): fusion across statements, which the backend
decides per kernel, would let the same collision code round differently in different kernels
(the forward step and the reverse pass's replays of it must agree bit for bit).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbrb.so")
SOURCES = [os.path.join(HERE, "csrc", n)
           for n in ("lbrb_kernels.hip", "lbrb_adjoint.hip", "lbrb_walls.hip", "lbrb_analysis.hip",
                     "lbrb_construct.hip", "lbrb_noalloc.hip", "lbrb_plan.cpp", "lbrb_api.cpp")]
ARCH = os.environ.get("LBRB_ARCH", "gfx950")


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False, extra=()) -> str:
    out = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
           "-o", out] + list(extra) + SOURCES + [
               "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs:
        print(msgs)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
