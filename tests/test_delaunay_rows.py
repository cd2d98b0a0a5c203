"""Host check of the prior's device triangulation rules (lf_delaunay.h and the
flip rounds of lf_prior.hip, replayed one round at a time): the row strips
and side pockets tile the frame, and the flips end at a Delaunay
triangulation, on random point sets laid out as the prior's."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_row_triangulation_and_flip_rounds(tmp_path):
    exe = tmp_path / "dt_rows_check"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "dt_rows_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok "), out.stdout
