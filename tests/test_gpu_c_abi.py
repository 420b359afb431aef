"""A plain C program using the library through include/gks.h only (no
Python in the loop): tests/c_abi/sine_c.c, built by __graft_entry__.build()."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "sine_c")


def test_c_program_runs_the_sine_wave_period():
    assert os.path.exists(EXE), "tests/c_abi/sine_c is not built (run __graft_entry__.build())"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "rejected: problem 0: order must be 6 or 8" in r.stdout
    assert "t = 2 after" in r.stdout and "status 1" in r.stdout
