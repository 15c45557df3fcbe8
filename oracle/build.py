"""Build the C oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, -O2 with floating-point contraction disabled so that every
multiply and add rounds separately, libm transcendentals, OpenMP only for the
loop over independent systems.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source built with AddressSanitizer and UndefinedBehaviorSanitizer
# (every report fatal), for a CPU test run of the oracle's pins; the process
# loading it needs the ASan runtime preloaded (LD_PRELOAD)
LIB_SANITIZED = os.path.join(HERE, "liboracle_san.so")
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SANITIZED if sanitize else LIB
    opt = SANITIZE_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc", "-std=c11", *opt, "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
