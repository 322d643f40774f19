"""Host unit test of the scheduler's arena allocator (C++, g++ here, no GPU):
tests/cpp/test_arena.cpp drives pd_arena.hpp against a brute-force model."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_first_fit_against_brute_force(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "test_arena"
    cmd = [cxx, "-O1", "-std=c++17", "-Wall", "-Werror",
           "-I" + os.path.join(ROOT, "paper_2006_09808_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "test_arena.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, timeout=120)
    p = subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True, timeout=120)
    assert p.returncode == 0, p.stdout
    assert p.stdout.startswith("ok ")
