"""The host BVH builder under the address and undefined-behaviour sanitizers
(g++), checked for the structure of its output (tests/native/bvh_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_bvh_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "bvh_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-pthread", "-o", exe,
           os.path.join(ROOT, "tests", "native", "bvh_check.cpp"),
           os.path.join(ROOT, "paper_1811_03510_amd", "csrc", "bvh_build.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "0 failure(s)" in r.stdout and "runtime error" not in r.stderr
