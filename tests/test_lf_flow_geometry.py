"""CPU check of the waits of the persistent lagged-Fibonacci LD run (paper_1003_1123_amd/csrc/lf_flow.hpp):
the waits against brute force, and a simulation of the whole producer/consumer protocol under random
interleavings (every read finds its position, every value equals the sequential recurrence, no
deadlock).  Compiled with the host compiler."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_waits_and_protocol_simulation():
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "lf_flow_check")
        subprocess.check_call([cxx, "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "native", "lf_flow_check.cpp")])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout
