"""The host conversion code (convert.cpp, features.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: a C++ driver built with g++ (host code only, no device code) runs
the planning, conversion, column-split, ELLPACK-R and feature entry points on ragged seeded
matrices and on invalid input, checking the format's invariants.  Any sanitizer report or
failed check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1112_5588_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_conversion_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    build = ["g++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-pthread",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             f"-I{os.path.join(ROOT, 'include')}", os.path.join(CSRC, "convert.cpp"), os.path.join(CSRC, "features.cpp"),
             os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1",
               PJDS_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "0 failures" in r.stdout
