"""The CPU-side code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle (all of it) and the library's host code (argument checks, planning, workspace
layout) are rebuilt with both sanitizers, and the oracle pins and the host-side ABI tests
run against those builds in a child process with the sanitizer runtime preloaded; any
report (out-of-bounds access, use after free, undefined behaviour) ends the child with an
error.  No device is used: the host ABI tests stop at argument checking."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_suites_under_sanitizers(tmp_path):
    from paper_2604_15645_amd import build
    from oracle import oracle
    rt = build.asan_runtime()
    if rt is None or not os.path.exists(oracle.CLANG):
        pytest.skip("no clang sanitizer runtime")
    if not os.path.exists(os.path.join(ROOT, "_build", "pinn_api.cpp.o")):
        pytest.skip("the library has not been built here (build() first)")
    lib = build.build_host_asan()
    olib = oracle.build_sanitized(str(tmp_path))
    # reports go to files: the child's pytest captures its own stderr
    logs = tmp_path / "reports"
    logs.mkdir()
    env = dict(os.environ, LD_PRELOAD=rt, PINN_LIB=lib, PINN_ORACLE_LIB=olib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:log_path=%s" % (logs / "asan"),
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:log_path=%s" % (logs / "ubsan"))
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_abi_host.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = "".join(f.read_text()[-3000:] for f in sorted(logs.iterdir()))
    tail = reports + (r.stdout + r.stderr)[-2000:]
    assert r.returncode == 0 and not reports, tail
    assert " passed" in r.stdout, tail
