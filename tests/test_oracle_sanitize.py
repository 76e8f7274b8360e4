"""Every oracle entry point once under AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code; oracle/sanitize_main.c): a
memory error or undefined behaviour anywhere in the oracle fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OR = os.path.join(ROOT, "oracle")


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "orc_san")
    srcs = [os.path.join(OR, f) for f in ("sanitize_main.c", "oracle.c", "mpnn.c", "vv.c", "block.c")]
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", exe] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "ok" in res.stdout
