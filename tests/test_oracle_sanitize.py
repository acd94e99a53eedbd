"""The oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host only) and run over exhaustive and random pins by a C driver that
compares every labeling with a textbook flood fill."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-std=c11", "-pthread", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", str(exe),
           os.path.join(ROOT, "oracle", "ccl_oracle.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")]
    subprocess.run(cmd, check=True)
    # (verify_asan_link_order=0: the sanitizer runtime tolerates libraries
    # that the environment loads ahead of it)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "0 failures" in res.stdout
