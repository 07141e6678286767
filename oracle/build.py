"""Build the oracle shared library (plain C, gcc, no contraction, no fast-math).

Test infrastructure: the product path never loads this library."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["elem.c", "model_real.c", "model_cplx.c", "setup.c", "assemble.c", "grad.c"]
OUT = os.path.join(HERE, "_build", "liboracle.so")


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fexcess-precision=standard", "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", OUT] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
