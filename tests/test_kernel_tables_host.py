"""Selector tables of the kernels (4x4 block permutes of the rotation, the
4-pixel field permutes of data hiding, the glide fill), checked on the
host with a CPU model of the byte-permute instruction (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_perm4_tables(tmp_path):
    exe = tmp_path / "perm4_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-o", str(exe), os.path.join(HERE, "host", "perm4_check.cpp")],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "cases 1024 mismatches 0" in out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_hide4_tables(tmp_path):
    exe = tmp_path / "hide4_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-o", str(exe), os.path.join(HERE, "host", "hide4_check.cpp")],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_glide4_tables(tmp_path):
    exe = tmp_path / "glide4_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-o", str(exe), os.path.join(HERE, "host", "glide4_check.cpp")],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "cases 1024 mismatches 0" in out.stdout
