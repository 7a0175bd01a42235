"""The library's host-only code (csrc/host.cpp: lattice tables, argument
checks, checkpoint header checks, layout rearrangement, tune cache) built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, no GPU code) and run over
synthetic inputs by tests/host_sanitize_driver.cpp: no out-of-bounds access,
leak or undefined operation."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_02503_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitized")
    build = ["g++", "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{CSRC}",
             os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), os.path.join(CSRC, "host.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host sanitizer driver: ok" in r.stdout
    assert "runtime error" not in r.stderr
