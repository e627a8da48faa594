"""Builds the CPU oracle library (test infrastructure only).

    python oracle/build.py

Compiles mem_oracle.c with gcc into oracle/liborc.so.  No multiply-add
contraction and no fast-math: the binary32 decision formulas must evaluate
exactly as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, f) for f in ("mem_oracle.c", "unet_oracle.c")]
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
