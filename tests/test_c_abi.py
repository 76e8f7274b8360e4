"""The library through its C ABI alone: tests/c_abi/step_demo.c includes
include/sim.h, links libsim.so with gcc and checks properties that hold for
any data (positions stay in the box, the step counter, sum_i v_i =
sum_i b_i / gamma0 for a solve, since 1^T A = gamma0 1^T, and the rejection
of gamma0 = 0)."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "c_abi"))
import build as c_build  # noqa: E402

BIN = os.path.join(HERE, "c_abi", "step_demo")


def test_demo_compiles_and_links(tmp_path):
    out = c_build.build(out=str(tmp_path / "step_demo"))
    assert os.path.exists(out)


@pytest.mark.gpu
def test_demo_runs():
    assert os.path.exists(BIN), "build first: python -c 'import __graft_entry__ as g; g.build()'"
    res = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "c abi ok" in res.stdout
