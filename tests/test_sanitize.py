"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/helpers/oracle_sanitize.c calls every oracle entry point (walk in
both start readings, index, top-k with padded rows, features, kNN within
and across graphs, walk_pids past 2^40, streamed counts, sample size,
rejected inputs) on a small graph with an isolated vertex and a zero-weight
edge.  It is compiled together with oracle/oracle.c by gcc with the
sanitizers (no OpenMP, so the runtime sees plain loops) and must print "ok"
with no report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "helpers", "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
