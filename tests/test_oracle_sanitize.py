"""The oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host only) and run on small pencils by tests/oracle_sanitize_driver.c:
out-of-bounds accesses, leaks, use after free or undefined arithmetic in any of
its routines fail this test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off",
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    # verify_asan_link_order=0: the run environment may preload libraries of its own
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "sanitized oracle run ok" in r.stdout
