"""Compile the FP64 oracle (``hs_oracle.c``) into ``oracle/libhs_oracle.so``.

Test infrastructure only: the HIP library never links or loads this file.
Plain gcc, OpenMP over independent output rows, no vector intrinsics.

``build(out=..., cc=..., extra=...)`` writes a variant elsewhere with another
compiler and extra flags (the sanitized copy of the CPU test-suite); the
arithmetic flags are the same in every build.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hs_oracle.c")
LIB = os.path.join(HERE, "libhs_oracle.so")


# -O2 without -ffast-math: IEEE double arithmetic in source order.
# -ffp-contract=off keeps a*b+s as two rounded operations (no FMA fusion),
# so every element is the plain ascending-k sum of rounded products.
ARITH_FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True, out: str = None, cc: str = "gcc", extra=("-fopenmp",)) -> str:
    target = out or LIB
    if not force and os.path.exists(target) and os.path.getmtime(target) >= os.path.getmtime(SRC):
        return target
    subprocess.check_call([cc] + ARITH_FLAGS + list(extra) + ["-o", target + ".tmp", SRC, "-lm"])
    os.replace(target + ".tmp", target)
    return target


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
