"""Host level builders under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): tests/host_setup_check.cpp is compiled with g++ against the
library's host_setup.cpp and run; it checks CSR patterns, patch maps and
their transpose, transfer stencils (Taylor-Hood and heat P_k) and the slab
integration-by-parts identity of the temporal tables for q = 0..3."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_setup_under_sanitizers():
    src = os.path.join(ROOT, "paper_2407_13997_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "host_setup_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-I", src, os.path.join(ROOT, "tests", "host_setup_check.cpp"),
               os.path.join(src, "host_setup.cpp"), "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "0 failures" in r.stdout
