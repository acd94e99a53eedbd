"""The threaded PARemSP of the oracle (POSIX threads, boundary unions under
Algorithm 8's locks) built with ThreadSanitizer (gcc, host only) and run by a
C driver that compares every result with single-threaded CCLRemSP."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_threaded_paremsp_under_thread_sanitizer(tmp_path):
    exe = tmp_path / "oracle_tsan"
    cmd = ["gcc", "-std=c11", "-pthread", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=thread", "-o",
           str(exe), os.path.join(ROOT, "oracle", "ccl_oracle.c"), os.path.join(ROOT, "tests", "sanitize",
                                                                               "tsan_driver.c")]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert "ThreadSanitizer" not in res.stderr, res.stderr[-4000:]
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    assert " 0 failures" in res.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_thread_sanitizer_sees_a_planted_race(tmp_path):
    """The same run on a copy of the oracle whose parent entries are read and
    written plainly (no atomics) must be reported as a data race: the check
    above is only worth something if it can fail."""
    src = open(os.path.join(ROOT, "oracle", "ccl_oracle.c")).read()
    old_ld = "    return __atomic_load_n(&p[i], __ATOMIC_RELAXED);"
    old_st = "    __atomic_store_n(&p[i], v, __ATOMIC_RELAXED);"
    assert src.count(old_ld) == 1 and src.count(old_st) == 1
    mut = tmp_path / "racy.c"
    mut.write_text(src.replace(old_ld, "    return p[i];").replace(old_st, "    p[i] = v;"))
    exe = tmp_path / "racy_tsan"
    subprocess.run(["gcc", "-std=c11", "-pthread", "-O1", "-g", "-fsanitize=thread", "-o", str(exe), str(mut),
                    os.path.join(ROOT, "tests", "sanitize", "tsan_driver.c")], check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode != 0 and "data race" in res.stderr
