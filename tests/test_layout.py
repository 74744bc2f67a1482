"""The storage layout's index arithmetic, checked on the host: the functions the
kernels use (lsmg_dev.hpp) compiled into a host program with hipcc and run on the
CPU (tests/layout/check_layout.cpp), for the compiled brick shape and for every
other 32-value shape the layout allows."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "layout", "check_layout.cpp")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("shape", [None, (3, 1), (1, 2), (2, 1), (1, 1)])
def test_storage_index_arithmetic(tmp_path, shape):
    exe = str(tmp_path / "check_layout")
    cmd = [HIPCC, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_1902_07029_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), SRC, "-o", exe]
    if shape:
        cmd[1:1] = [f"-DLSMG_BRICK_P={shape[0]}", f"-DLSMG_BRICK_J={shape[1]}"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
