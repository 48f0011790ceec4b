"""Host code under AddressSanitizer and UBSan (CPU only): the FP64 oracle's
C entry points and libplbm's host layer (coefficients, descriptor defaults,
validation, sizes), each built with gcc / g++ and run by a small driver on
valid, degenerate and hostile inputs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
       "-fno-sanitize-recover=all"]


def _build_and_run(compiler, sources, out, extra=()):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    cmd = [compiler, *SAN, *extra, *sources, "-o", out, "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    r = subprocess.run([out], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    _build_and_run("gcc", [os.path.join(ROOT, "tests", "asan", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "ref_plbm.c")],
                   str(tmp_path / "oracle_asan"))


def test_library_host_layer_under_address_and_ub_sanitizers(tmp_path):
    _build_and_run("g++", [os.path.join(ROOT, "tests", "asan", "host_driver.cpp"),
                           os.path.join(ROOT, "paper_1402_5487_amd", "csrc", "plbm_coeffs.cpp")],
                   str(tmp_path / "host_asan"),
                   extra=("-std=c++17", "-I", os.path.join(ROOT, "include"),
                          "-I", os.path.join(ROOT, "paper_1402_5487_amd", "csrc")))
