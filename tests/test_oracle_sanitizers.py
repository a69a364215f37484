"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): every variant of a whole run on small grids, including the
paranoid recomputation mode, ends cleanly."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "orc_san")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "mpma_oracle.c"),
           os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True)
    if r.returncode != 0 and b"asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr.decode()
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, env=env, timeout=240)
    assert r.returncode == 0, (r.stdout + r.stderr).decode()[-2000:]
    assert b"ok" in r.stdout
