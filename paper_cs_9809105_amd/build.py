"""Build the C-ABI library ``libhs.so`` (HIP kernels for gfx950 + host API).

    python -m paper_cs_9809105_amd.build [--verbose]

Compiles in-tree with hipcc; the result sits next to this file so that it
travels with the source tree.  Every build recompiles.

``build(out=..., extra=...)`` writes a variant elsewhere with extra flags
(the sanitized copy of the CPU test-suite); the product library is always
``libhs.so`` beside this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhs.so")
SOURCES = [os.path.join(CSRC, "hs_kernels.hip"), os.path.join(CSRC, "hs_nbody.hip"),
           os.path.join(CSRC, "hs_api.cpp"), os.path.join(CSRC, "hs_noalloc.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False, extra=(), out=None):
    target = out or LIB
    tmp = target + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra) + SOURCES + ["-o", tmp]
    if verbose:
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    log = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + log)
    os.replace(tmp, target)
    if verbose and log.strip():
        print(log)
    return target


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
