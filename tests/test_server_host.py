"""Host-only bookkeeping of the server and of run results (no GPU): the
first-fit arena against a granule model, and result sizing from the
device's count of generations run, built with AddressSanitizer and
UndefinedBehaviorSanitizer."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(not shutil.which("g++"), reason="g++ missing")
@pytest.mark.parametrize("sanitize", [False, True])
def test_server_bookkeeping(tmp_path, sanitize):
    exe = tmp_path / "server_host_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", os.path.join(HERE, "server_host_check.cpp"),
           "-o", str(exe)]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.check_call(cmd)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr
