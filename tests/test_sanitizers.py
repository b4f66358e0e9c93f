"""The oracle and the host-side argument checks of the C ABI, built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, CPU only) and run on
small, degenerate and extreme inputs by the harnesses in tests/sanitize/."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("the compiler has no sanitizer runtime here")
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_harness")
    _build(["gcc", *SAN, "-fopenmp", "-std=c11", os.path.join(ROOT, "tests/sanitize/oracle_harness.c"),
            os.path.join(ROOT, "oracle/lfbp_oracle.c"), "-o", exe, "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_argument_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "validate_harness")
    _build(["g++", *SAN, "-std=c++17", "-I" + os.path.join(ROOT, "include"),
            "-I" + os.path.join(ROOT, "paper_2003_09133_amd/csrc"),
            os.path.join(ROOT, "tests/sanitize/validate_harness.cpp"),
            os.path.join(ROOT, "paper_2003_09133_amd/csrc/lfbp_validate.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
