"""Compile the FP64 oracle (``hs_oracle.c``) into ``oracle/libhs_oracle.so``.

Test infrastructure only: the HIP library never links or loads this file.
Plain gcc, OpenMP over independent output rows, no vector intrinsics.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hs_oracle.c")
LIB = os.path.join(HERE, "libhs_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    # -O2 without -ffast-math: IEEE double arithmetic in source order.
    # -ffp-contract=off keeps a*b+s as two rounded operations (no FMA fusion),
    # so every element is the plain ascending-k sum of rounded products.
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
