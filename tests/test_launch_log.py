"""Host logic of the profiling window (csrc/launch_log.hpp), built with the
host compiler and run on the CPU: a launch that fails after reserving its
event pair leaves no record and frees the pair, so the events of every
record bracket exactly its own launch."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_launch_log_pairs_events_with_their_launches(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "launch_log_check"
    src = os.path.join(ROOT, "tests", "csrc", "launch_log_check.cpp")
    inc = os.path.join(ROOT, "paper_2507_03509_amd", "csrc")
    subprocess.run([cxx, "-std=c++17", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    f"-I{inc}", src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"
