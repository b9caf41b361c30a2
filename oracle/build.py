"""Build the CPU oracle shared library (test infrastructure only).

``python -m oracle.build`` compiles ``oracle/oracle.c`` into
``oracle/liboracle.so`` with gcc: long double arithmetic, OpenMP over seeds and
starting points, ``-frounding-math`` so that the round-upward certificate
passes are not reordered, and no floating-point contraction.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = [
    "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
    "-frounding-math", "-ffp-contract=off", "-fno-fast-math",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
