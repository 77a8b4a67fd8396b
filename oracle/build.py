"""Compile the oracle's C sources into ``oracle/liborc.so`` with gcc (-O2, OpenMP, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  No -ffast-math: the oracle keeps
IEEE semantics so its arithmetic follows the source order.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_lattice.c", "orc_philox.c", "orc_lbrb.c", "orc_adjoint.c", "orc_relax.c"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
