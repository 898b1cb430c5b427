"""The C ABI used from C: the example program builds against include/cvo.h
and the library alone (no Python in the process), recovers its motion, and
gets the same result bit for bit from four tickets of the scheduler."""
import math
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_c_example_registers(tmp_path):
    exe = str(tmp_path / "register_planes")
    lib = os.path.join(ROOT, "paper_1904_02266_amd", "lib")
    subprocess.run(["gcc", "-O2", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "paper_1904_02266_amd", "examples", "register_planes.c"),
                    "-L", lib, "-lcvo", "-lm", "-Wl,-rpath," + lib, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    m = re.search(r"rotation about z (\S+) deg translation (\S+) (\S+) (\S+)", out.stdout)
    ang, tx, ty, tz = (float(v) for v in m.groups())
    a = math.radians(3.0)
    R = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    t_inv = -R.T @ np.array([0.03, -0.02, 0.01])
    assert abs(ang + 3.0) < 0.05, out.stdout
    assert np.linalg.norm(np.array([tx, ty, tz]) - t_inv) < 0.003, out.stdout
    assert "served 4 of 4 equal to the synchronous result; completed 4 failed 0" in out.stdout, out.stdout
