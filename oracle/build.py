"""Compile the oracle's C table routine (oracle/pbar.c) into oracle/libpbar.so.

TEST INFRASTRUCTURE: the library is loaded only by the oracle (tests, smoke check, the
benchmark's CPU-baseline leg).  Plain IEEE FP64: no fast-math, no FMA contraction.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pbar.c")
LIB = os.path.join(HERE, "libpbar.so")


def build(verbose=False):
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
