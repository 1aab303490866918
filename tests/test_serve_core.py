"""CPU test of the serving bookkeeping (pool carving, admission with bounded
bypass, failed launches, cancellation): the header the server is built from,
compiled with the host compiler and driven with simulated completions."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_serve_core(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "serve_core_check"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I",
                    os.path.join(ROOT, "paper_1607_07395_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "serve_core_check.cpp"), "-o", str(exe)],
                   check=True)
    p = subprocess.run([str(exe)], capture_output=True, text=True)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "all ok" in p.stdout
