"""The render server's scheduler, on the CPU with a fake executor, built with
g++ plain and under ThreadSanitizer and AddressSanitizer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "serve_core_test.cpp")
INC = os.path.join(ROOT, "paper_2103_10380_amd", "csrc")


@pytest.mark.parametrize("san", ["", "thread", "address"])
def test_scheduler(tmp_path, san):
    exe = str(tmp_path / f"serve_core_test_{san or 'plain'}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I" + INC, SRC, "-o", exe]
    if san:
        cmd.insert(1, f"-fsanitize={san}")
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all tests passed" in r.stdout
