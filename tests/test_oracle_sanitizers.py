"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host only) and driven through every exported function on the four
parameter sets and on edge inputs (tests/sanitize_oracle.c): no invalid
access, leak or undefined arithmetic."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "ntrup_oracle.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(HERE, "sanitize_oracle.c"), SRC, "-o", exe])
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok"), out.stdout
    assert "runtime error" not in out.stderr, out.stderr
