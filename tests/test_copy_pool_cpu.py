"""Host-only check of the copy pool that moves pageable caller memory
through page-locked staging in the host-memory pipeline: compiled with g++
from the library's header (no device code), every byte of every copy must
arrive and nothing past the end may be written."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_copy_pool_covers_every_byte(tmp_path):
    exe = tmp_path / "copy_pool_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread",
                    "-I", os.path.join(ROOT, "paper_2204_02085_amd", "csrc"),
                    os.path.join(ROOT, "tests", "copy_pool_check.cpp"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "copy pool ok" in out.stdout
