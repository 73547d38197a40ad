"""The oracle's C solvers under gcc's address and undefined-behaviour sanitizers (CPU only): oracle/solvers.c
linked with its stand-alone check oracle/solvers_selfcheck.c, which compares both solvers with brute force on
seeded random problems of up to 12 nodes (half of them tie-prone) and exits non-zero on the first mismatch or
sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_solvers_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_selfcheck")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Werror",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", exe, os.path.join(ORACLE, "solvers_selfcheck.c"), os.path.join(ORACLE, "solvers.c")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "3000"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok 3000"
