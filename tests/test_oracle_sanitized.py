"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) and run through every function on small stored-cost and
fused-cost problems (tests/oracle_sanitize_driver.c): no out-of-bounds
access, leak or undefined behaviour is reported."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", exe, os.path.join(HERE, "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "srot_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=240)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    assert res.stdout.strip() == "ok"
    assert "runtime error" not in res.stderr, res.stderr[-4000:]
