"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, g++), driven through every exported routine by
oracle/sanitize_main.cpp: any out-of-bounds access, use after free, leak or
undefined operation makes the driver exit non-zero.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
@pytest.mark.skipif(not shutil.which("g++"), reason="g++ not available")
@pytest.mark.skipif(bool(os.environ.get("LD_PRELOAD")), reason="a preloaded library would precede the sanitizer runtime")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", str(exe), os.path.join(ROOT, "oracle", "sanitize_main.cpp"), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "checksum" in r.stdout
