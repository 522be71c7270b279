"""Compile the FP64 oracle (plain C, OpenMP) into oracle/liboracle.so.

Test infrastructure: the library built here is the checker, never a compute
path of the package.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# -ffp-contract=off keeps every FP64 operation a separately rounded one, so
# the oracle gives the same bits on any x86-64 host.
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    cc = os.environ.get("CC", "gcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc] + CFLAGS + [SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
