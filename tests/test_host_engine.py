"""The library's host-side numerics (window series and table, Gauss-Legendre
rules, I0, neighbour ranges, the upper ranges of the pair-once local sum)
built with AddressSanitizer and UndefinedBehaviorSanitizer and checked on the
CPU (tests/host/host_checks.cpp): brute force for the ranges, exactness and
closed-form values for the rest."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_engine_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(HERE, "host", "host_checks.cpp"),
           os.path.join(ROOT, "paper_2507_07823_amd", "csrc", "wfp_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host checks passed" in r.stdout
