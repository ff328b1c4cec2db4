"""The traversal's launch geometry (csrc/launch_geometry.h), compiled with g++
on the CPU: for systems of several types, the workgroups the host launches
hold every wavefront the device maps queries to, and the eight stretches
cover every query of every type exactly once (300k random type splits, every
workgroup width and queries-per-wavefront setting)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_launch_geometry(tmp_path):
    exe = tmp_path / "launch_geometry_test"
    src = os.path.join(HERE, "launch_geometry_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", src, "-o", str(exe)], check=True)
    proc = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert proc.returncode == 0, proc.stdout + proc.stderr
    assert "all checks passed" in proc.stdout
