"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/oracle_asan_driver.c calls every oracle entry point (all schemes, a
registered scheme, both boundary rules and first steps, grids down to 3 x 3
and too small for the periodic 13-point rule) on exactly sized allocations;
the build aborts at the first out-of-bounds access or undefined operation.
Host code only (gcc); OpenMP off so the sanitizer sees one thread.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "wave2d_oracle.c"), os.path.join(HERE, "oracle_asan_driver.c"),
           "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr
    assert "runs" in out.stdout
