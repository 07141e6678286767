"""Build libcolorstamp.so for gfx950 in-tree (hipcc; no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_lib", "libcolorstamp.so")
SOURCES = ["kernels.hip", "adjoint.hip", "setup.cpp", "region.cpp", "api.cpp", "batch.cpp", "sparse_lu.cpp",
           "newton.cpp", "solve.hip", "tune.cpp", "noalloc.hip"]
# the Newton loop's sparse refactorisation and triangular solves
LIBS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocsolver", "-lrocblas"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # bit-exact FP64: no contraction, no fast-math
    "-ffp-contract=off", "-fno-fast-math",
    # hardware FP64 atomic add for the atomic variant
    "-munsafe-fp-atomics",
    # packed FP32 instructions off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    cmd = ["/opt/rocm/bin/hipcc"] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                             "-o", OUT + ".tmp"] + srcs + LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs.strip():
        print(msgs)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
