"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's host CSR builder and the C oracle, driven by
tests/sanitize/host_driver.cpp over seeded random inputs and error paths."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_builder_and_oracle_clean_under_sanitizers(tmp_path):
    oracle_o = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", *SAN, "-std=c99", "-c", os.path.join(ROOT, "oracle", "ktruss_oracle.c"), "-o", oracle_o],
                   check=True)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                    os.path.join(ROOT, "paper_2009_07929_amd", "csrc", "csr_build.cpp"), oracle_o, "-o", exe],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitizer harness ok" in r.stdout
