"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc), driven by tests/sanitize_oracle.c through its tracker with a work crew
of threads, the duplicate scan, the double-double end game, the LU solve and
the predictor: the run must finish cleanly (no invalid access, leak or
undefined operation reported)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-pthread",
           os.path.join(HERE, "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    # a library preloaded into every process would otherwise precede the
    # sanitizer runtime in the link order, which it checks by default
    env["ASAN_OPTIONS"] = "detect_leaks=1:verify_asan_link_order=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "converged 12 of 12" in r.stdout
