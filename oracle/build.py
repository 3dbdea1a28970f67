"""Compile the CPU oracle (test infrastructure) into oracle/_gs_oracle.so with gcc + OpenMP.

The FP32 binning file is compiled without FMA contraction so its float32 decisions follow
the operation order written in it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "_gs_oracle.so")
SOURCES = ["gs_oracle.c", "bins32.c"]


FLAGS = ["-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-D_DEFAULT_SOURCE"]
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2"] + FLAGS + ["-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The same sources with AddressSanitizer and UndefinedBehaviorSanitizer (any report is
    fatal), for loading into a process that preloads gcc's libasan and libubsan."""
    cmd = ["gcc", "-O1"] + FLAGS + SANITIZE + ["-o", out] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
