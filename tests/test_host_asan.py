"""The host code builder under AddressSanitizer and UndefinedBehaviorSanitizer.

g++ compiles the builder (paper_1711_01783_amd/csrc/met_code.cpp, host C++ only)
with both sanitizers, together with tests/asan_builder.cpp, which drives every
construction path, the derived decoder structures and the validation errors.
Any out-of-bounds access, use after free, leak or undefined operation aborts the
program and fails the test.  No GPU code is built.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_builder_clean_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "asan_builder")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1711_01783_amd", "csrc"),
           os.path.join(ROOT, "tests", "asan_builder.cpp"),
           os.path.join(ROOT, "paper_1711_01783_amd", "csrc", "met_code.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    # verify_asan_link_order=0: the environment may preload another library
    # ahead of the sanitizer runtime; that does not change what is checked
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "asan builder ok" in r.stdout
