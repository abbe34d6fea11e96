"""The serving scheduler's admission, arena and tick logic (C++ header used
by the server), exercised on the CPU with a fake device by a C++ test
program built here with address and undefined-behaviour sanitizers."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_server_core(tmp_path):
    exe = tmp_path / "test_server_core"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                           os.path.join(HERE, "cpp", "test_server_core.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
