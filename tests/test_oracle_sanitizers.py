"""The CPU oracle under gcc's address and undefined-behaviour sanitizers:
tests/oracle_sanitize_main.c drives every code path (jumps, Bjorken table
with a thermal shift and derivType 1, a kappa_hat fit, maxJumps with strided
ids, rMax, the no-jump shortcut, a vacuum phase, the kinetic-off flag, the
KSU potential, an empty run, the sine transform) with every output present.
Any out-of-bounds access, leak, overflow or other undefined behaviour aborts
the program."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + ORACLE, os.path.join(HERE, "oracle_sanitize_main.c"),
           os.path.join(ORACLE, "qtraj_oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 11, r.stdout
    assert all("rc=0" in line for line in lines[:-1])
