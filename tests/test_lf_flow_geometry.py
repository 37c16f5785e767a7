"""CPU check of the tile-dependency geometry of the dataflow lagged-Fibonacci LD kernel
(paper_1003_1123_amd/csrc/lf_flow.hpp) against brute force; compiled with the host compiler."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_tile_sources_match_brute_force():
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "lf_flow_check")
        subprocess.check_call([cxx, "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "native", "lf_flow_check.cpp")])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout
