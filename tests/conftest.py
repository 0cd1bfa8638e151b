import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The sanitized CPU run (tests/test_sanitizers.py) points the suite at
# instrumented copies of the two libraries through these variables.
SAN_LIBHS = os.environ.get("HS_TEST_LIBHS")
SAN_ORACLE = os.environ.get("HS_TEST_ORACLE_LIB")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    if SAN_LIBHS:
        from paper_cs_9809105_amd import binding
        binding.LIB_PATH = SAN_LIBHS
    if SAN_ORACLE:
        from oracle import build
        build.LIB = SAN_ORACLE


def pytest_report_header(config):
    if SAN_LIBHS or SAN_ORACLE:
        return "sanitized libraries: libhs=%s oracle=%s" % (SAN_LIBHS, SAN_ORACLE)


def pytest_sessionfinish(session, exitstatus):
    if SAN_LIBHS or SAN_ORACLE:
        with open("/proc/self/maps") as f:
            maps = f.read()
        loaded = [p for p in (SAN_LIBHS, SAN_ORACLE) if p and p in maps]
        print("\n[sanitize] asan runtime mapped: %s; loaded: %s"
              % ("libclang_rt.asan" in maps, " ".join(loaded)))
