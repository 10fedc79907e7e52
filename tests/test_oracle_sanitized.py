"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) runs every entry point over small lattices of each model
without a report: no access outside its arrays, no overflow of signed
arithmetic, no invalid shift, no leak."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not on PATH")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "swo_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "sw_oracle.c"),
           "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr + b.stdout).lower():
        pytest.skip("this gcc has no sanitizer runtime: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and "oracle sanitize: ok" in r.stdout, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
