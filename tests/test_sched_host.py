"""The scheduler of the C ABI (csrc/pd_host.cpp) on the CPU, without a GPU:
tests/cpp/sched_mock.cpp builds it with g++ against a host-only stand-in of
the HIP runtime and mock kernel launchers that count the iterations each
slice pair receives, then drives admission under a full arena, rounds with
gap-check stops, staggered arrivals, the recovery from a resident launch that
gives up, and pd_destroy while other threads wait in pd_poll.  Built twice:
with the address and undefined-behaviour sanitizers, and with the thread
sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_09808_amd", "csrc")


def _build_and_run(tmp_path, sanitize, name):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / name
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-pthread", "-fno-omit-frame-pointer",
           "-fsanitize=" + sanitize,
           "-I" + os.path.join(ROOT, "tests", "cpp", "mockhip"), "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, os.path.join(CSRC, "pd_host.cpp"), os.path.join(ROOT, "tests", "cpp", "sched_mock.cpp"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", TSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300,
                       env=env)
    print(p.stdout)
    assert p.returncode == 0, p.stdout[-4000:]
    assert "WARNING: ThreadSanitizer" not in p.stdout
    assert p.stdout.strip().splitlines()[-1].startswith("ok ")


def test_scheduler_mock_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, "address,undefined", "sched_mock_asan")


def test_scheduler_mock_tsan(tmp_path):
    _build_and_run(tmp_path, "thread", "sched_mock_tsan")
