"""The host-side math of libstig (quadrature, B-splines, assembly, separation,
eigensolvers, arrowhead factorization) built for the CPU with AddressSanitizer
and UndefinedBehaviorSanitizer and run on the identities it must satisfy
(tests/host_math_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_math_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_math_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "tests", "host_math_check.cpp"),
           os.path.join(ROOT, "paper_1909_07309_amd", "csrc", "host_math.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "host math ok" in r.stdout
