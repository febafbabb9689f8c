"""Host sanitizers on the FP64 oracle: tests/oracle_sanitize_driver.c is
built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, single
thread) and must run clean."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_asan"
    cmd = ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(HERE, "oracle_sanitize_driver.c"), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
