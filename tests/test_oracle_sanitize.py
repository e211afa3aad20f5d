"""The CPU oracle built with the address and undefined-behaviour sanitizers
(gcc) and driven over every entry point, format, mode, operation and flag on
small inputs: no memory error, no undefined behaviour, every call returns
its expected status."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_exercise")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I" + os.path.join(ROOT, "oracle"), os.path.join(HERE, "sanitize", "oracle_exercise.c"),
           os.path.join(ROOT, "oracle", "mxfft_oracle.c"), "-o", exe, "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle exercise: ok" in r.stdout
