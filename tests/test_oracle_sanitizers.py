"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/brng_oracle.c is the one C component that runs here; a driver
(tests/oracle_sanitize_driver.c) calls each of its exported functions on
small ragged inputs (partial units, items of 0 to 300 components, invalid
parameters) with buffers of exact size, built with gcc's address,
undefined-behaviour and float-cast-overflow checks, every finding fatal.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize_driver")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc"] + flags + [os.path.join(HERE, "oracle_sanitize_driver.c"),
                                             os.path.join(ROOT, "oracle", "brng_oracle.c"),
                                             "-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "driver ok" in p.stdout
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr
