"""The selection phase's threshold rule with batched passes (the library's
host core, select_core.h) against the rule run one threshold per pass, on
synthetic cluster counts, compiled with the host compiler (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_select_core_matches_serial_rule(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "select_core_test"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    os.path.join(HERE, "select_core_test.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "select core ok" in r.stdout
