"""The CPU oracle under gcc's address and undefined-behaviour sanitizers:
its build (grid, sort, neighbour lists, B0, damping schedule), the lone
stepping pieces and the multi-time-step driver on small jittered lattices
(2D coupled diffusion with the mixture momentum, 2D loading with the
adaptive stop, 3D J2 into the plastic range), in the FP64 and in the
complex-step build.  Any out-of-bounds access, leak or undefined operation
ends the run with an error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sph_oracle.c")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("complex_step", [False, True], ids=["fp64", "complex"])
def test_oracle_runs_clean_under_sanitizers(tmp_path, complex_step):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), DRIVER, SRC, "-o", exe, "-lm"]
    if complex_step:
        cmd.insert(1, "-DORC_COMPLEX")
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout.split()
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
