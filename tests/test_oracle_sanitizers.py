"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle.c and a driver that calls every entry point on small problems
(tests/oracle_sanitize_driver.c) are built with gcc, the sanitizers on and
every finding fatal, and run; a memory error, a leak or undefined behaviour
fails the test.  Host code only (the GPU library is not built here).
"""
import os
import shutil
import subprocess

import pytest

from oracle import build as orabuild

TESTS = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wextra",
           "-Wno-unknown-pragmas", "-I" + os.path.dirname(orabuild.SRC),
           "-o", exe, os.path.join(TESTS, "oracle_sanitize_driver.c"), orabuild.SRC, "-lm"]
    subprocess.run(cmd, check=True)
    # verify_asan_link_order=0: the environment may preload a library of its own
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run ok" in r.stdout
