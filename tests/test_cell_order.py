"""Host check of the binning's cell order (paper_1309_1889_amd/csrc/common.h):
cell_rank is a bijection onto the cells, cell_coords inverts it, the 32-bit
form used by the pair search agrees with it, and consecutive bricks share a
face on domains of one strip of brick rows. The check program is built with
hipcc for the host only; it runs no GPU code."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cell_order_is_a_consistent_bijection(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "cell_order_check"
    subprocess.run([hipcc, "-O1", "-x", "hip", os.path.join(HERE, "cell_order_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.strip().splitlines()
    assert lines[-1] == "ok"
    for line in lines[:-1]:
        m = re.match(r"bricks (\d+) (\d+) (\d+): wrong (\d+), consecutive bricks not sharing a face (\d+)", line)
        assert m, line
        nb1 = int(m.group(2))
        assert int(m.group(4)) == 0, line
        # one strip (rows z after y over the whole domain): an unbroken snake
        if nb1 < 32:
            assert int(m.group(5)) == 0, line
