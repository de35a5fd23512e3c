"""Host code under AddressSanitizer and UBSan (CPU only): the layout builder
(csrc/layout.cpp) checked against brute force by tests/sanitized_layout_check.cpp,
and the C oracle by tests/sanitized_oracle_check.c.  Any invalid access,
undefined behaviour or leak ends the run with a report; a wrong table or value
fails the run's own checks."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2507_15121_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(cmd, exe):
    if shutil.which(cmd[0]) is None:
        pytest.skip("%s not found" % cmd[0])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, OMP_NUM_THREADS="4", UBSAN_OPTIONS="print_stacktrace=1",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-3000:] + r.stderr[-3000:])
    return r.stdout


def test_layout_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "layout_check")
    cmd = ["g++", "-std=c++17", "-fopenmp"] + SAN + [
        "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"), "-I" + CSRC,
        "-I" + os.path.join(ROOT, "include"),
        os.path.join(HERE, "sanitized_layout_check.cpp"), os.path.join(CSRC, "layout.cpp"), "-o", exe]
    out = _build_and_run(cmd, exe)
    assert "0 failures" in out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-std=c99"] + SAN + [
        os.path.join(HERE, "sanitized_oracle_check.c"), os.path.join(ROOT, "oracle", "mttkrp_ref.c"),
        "-lm", "-o", exe]
    out = _build_and_run(cmd, exe)
    assert "0 failures" in out
