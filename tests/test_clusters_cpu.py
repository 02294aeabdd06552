"""The diagonal grouping of the LDS-staged DIA sweep (pure host logic the
conversion uses), built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer: stencil, banded, scattered and random offsets."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_diagonal_clusters(tmp_path):
    exe = tmp_path / "clusters_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", str(exe), os.path.join(ROOT, "tests", "c", "clusters_driver.cpp")]
    subprocess.check_call(cmd)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "clusters driver ok" in r.stdout
