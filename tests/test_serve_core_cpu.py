"""The serving loop's host core (arena allocator + continuous-batching policy)
under a simulated executor, compiled with the host compiler (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_serve_core_invariants(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "serve_core_test"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    os.path.join(HERE, "serve_core_test.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "serve core ok" in r.stdout
