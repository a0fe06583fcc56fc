"""The host-only C++ of the library (validation of the topological assumptions of Sec. III-B,
the branch-list to mesh mapping of Sec. III eqs. 4-6, the colouring of general netlists) built
with AddressSanitizer and UndefinedBehaviorSanitizer and driven by tests/host/sanitize_driver.cpp:
seeded random meshes and their branch lists must map back exactly, colourings must separate every
coupled pair, corrupted inputs must be refused, and the sanitizers must report nothing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1409_7166_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp")] + \
    [os.path.join(CSRC, f) for f in ("validate.cpp", "netlist.cpp", "graph.cpp")]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), *SOURCES, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "2000"], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    words = r.stdout.split()
    assert "2000 round trips" in r.stdout and "2000 valid random graphs coloured" in r.stdout, r.stdout
    assert words[-3] == "0", r.stdout  # failed checks
