"""CPU check of the integer generator steps in paper_1003_1123_amd/csrc/gen_int.hpp: the Tausworthe
step's funnel-shift form against Eq. 2's shift-and-xor, its words against the component's bit
recurrence (Eq. 2), the LCG's n-step map against single steps, and the modular product of Ran2's
two generators against the 64-bit remainder.  Compiled with the host compiler."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_integer_generator_steps():
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "gen_int_check")
        subprocess.check_call([cxx, "-O2", "-std=c++17", "-Wall", "-Werror", "-o", exe,
                               os.path.join(HERE, "native", "gen_int_check.cpp")])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout
