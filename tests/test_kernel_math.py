"""The tabu-search kernel's pure integer helpers, compiled for the CPU.

Magic-number division (tenure, move-id decode), and the squeezed 16-bit move
scale of phase 2 with its aspiration bound (Section 3.3: aspiration admits a
tabu move that beats the phase's best).
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc missing")
def test_kernel_integer_helpers(tmp_path):
    exe = tmp_path / "kernel_math_check"
    src = os.path.join(HERE, "kernel_math_check.cpp")
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", src, "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout
