"""The server's admission and result-lifetime policy (csrc/server_core.h),
compiled with g++ on the CPU against a fake device and run as a program: a
published result is never overwritten while leased, eviction skips leased and
busy sessions, a request blocked by leased memory fails instead of waiting
forever, an idle lane's workspace is released when it blocks admission,
per-sim order and batching, allocation failure, cancellation and the bounded
latency window."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_server_core_policy(tmp_path):
    exe = tmp_path / "server_core_test"
    src = os.path.join(HERE, "server_core_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
                    "-fsanitize=address,undefined", src, "-o", str(exe)], check=True)
    proc = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert proc.returncode == 0, proc.stdout + proc.stderr
    assert "all checks passed" in proc.stdout
