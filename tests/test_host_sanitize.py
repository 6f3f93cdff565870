"""The host C++ of the library (plan-table builders, descriptor validation,
status strings, the host table export) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run over Yin-Yang and polar descriptors from
lmax 0 to 64, exact-size buffers and every invalid-descriptor case
(tests/native/host_checks.cpp).  Host code only: no HIP, no GPU."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_04593_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "native", "host_checks.cpp"),
           os.path.join(CSRC, "yyg_tables.cpp"), os.path.join(CSRC, "yyg_host.cpp"),
           "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, timeout=300)
    # the environment is passed on unchanged apart from the sanitizer
    # options (a library preloaded ahead of the ASan runtime is tolerated)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "host checks: 0 failures" in r.stdout
