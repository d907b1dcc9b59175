"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer: a driver runs
every oracle routine (validation, prefix products, root weights, alias table, sampling in IIS
and RIS mode from one preparation, transpose, estimates, greedy) on small random graphs and
checks invariants on the way; any out-of-bounds access, leak or undefined behaviour aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "ora_san")
    src = [os.path.join(ROOT, "oracle", "sanitize_check.c"), os.path.join(ROOT, "oracle", "skis_oracle.c")]
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-pthread", "-o", exe, *src, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "sanitized oracle run ok" in out.stdout
