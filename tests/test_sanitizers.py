"""The CPU test-suite again, under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds instrumented copies of libhs.so (host code: argument checks, plans,
workspace and 2^31 limits; the device code is unchanged) and of the FP64
oracle into a temporary folder, then runs every other ``-m "not gpu"`` test
in a child process with the clang ASan runtime preloaded and both copies
loaded in place of the plain builds (tests/conftest.py swaps the paths).
Any heap/stack overflow, use after free, signed overflow, invalid enum load,
misaligned or out-of-bounds access in either library aborts the child and
fails this test.  Leak checking is off: the interpreter is not instrumented.
The oracle copy is compiled by ROCm's clang (GNU OpenMP runtime) so that both
libraries share the one ASan runtime of the process.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import build as oracle_build  # noqa: E402
from paper_cs_9809105_amd import build as hs_build  # noqa: E402

CLANG = "/opt/rocm/llvm/bin/clang"
# hipcc: each sanitizer applies to the host pass only
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]
ORACLE_SANITIZE = ["-fopenmp=libgomp", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def asan_runtime():
    if not os.path.exists(CLANG):
        return None
    path = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                          stdout=subprocess.PIPE, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(bool(os.environ.get("HS_TEST_LIBHS")), reason="already the sanitized run")
def test_cpu_suite_under_asan_ubsan(tmp_path):
    runtime = asan_runtime()
    if runtime is None:
        pytest.skip("no clang ASan runtime in this image")
    libhs = hs_build.build(out=str(tmp_path / "libhs_san.so"), extra=HOST_SANITIZE)
    orac = oracle_build.build(out=str(tmp_path / "libhs_oracle_san.so"), cc=CLANG,
                              extra=ORACLE_SANITIZE)
    for lib, probe in ((libhs, "__asan_report_load8"), (libhs, "__ubsan_handle"),
                       (orac, "__asan_report_load8"), (orac, "__ubsan_handle")):
        syms = subprocess.run(["nm", "-D", lib], stdout=subprocess.PIPE, text=True).stdout
        assert probe in syms, "%s is not instrumented (%s)" % (lib, probe)
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime,
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "HS_TEST_LIBHS": libhs,
        "HS_TEST_ORACLE_LIB": orac,
    })
    # --capture=sys: a sanitizer report goes straight to the child's stderr
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-x",
           "-m", "not gpu", "-p", "no:cacheprovider", "--capture=sys",
           "--deselect", "tests/test_sanitizers.py::test_cpu_suite_under_asan_ubsan"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=900)
    tail = "\n".join(r.stdout.splitlines()[-40:])
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stdout and "runtime error:" not in r.stdout, tail
    assert "[sanitize] asan runtime mapped: True; loaded: %s %s" % (libhs, orac) in r.stdout, tail
    assert " passed" in r.stdout and " failed" not in r.stdout, tail
