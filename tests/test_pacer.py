"""Host pacing of the solver's step launches (csrc/pacer.h), compiled with
g++ and driven by a simulated device: even chunks (launch k has parity
k % 2), never more than the allowed chunks in flight or launches past the
limit, termination whenever the solve ends within the limit, and the idle
launches after the end bounded by the prediction margin (exact or long
prediction) or by the chunks in flight (none, or a short one)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2105_01586_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_pacer_properties(tmp_path):
    exe = str(tmp_path / "pacer_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC,
                    os.path.join(HERE, "pacer_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
