"""The host-side argument checks of the C ABI (csrc/gs_host.cpp: configuration, camera
tables, tile layout, status strings) built as a CPU program with the address and
undefined-behaviour sanitizers and driven with seeded random and boundary arguments
(tests/host_checks_main.cpp). No GPU is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2308_04079_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs the host C++ compiler")
def test_host_checks_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           os.path.join(CSRC, "gs_host.cpp"), os.path.join(ROOT, "tests", "host_checks_main.cpp"),
           "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "host checks ok" in run.stdout
