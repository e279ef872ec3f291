"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver (oracle/sanitize_main.c) calls every entry point on small cases, in
the plain and the complex-step build, compiled with gcc and both sanitizers
(any report aborts the run)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.parametrize("variant", ["plain", "complex_step"])
def test_oracle_clean_under_sanitizers(tmp_path, variant):
    exe = tmp_path / f"oracle_sanitized_{variant}"
    extra = ["-DOR_COMPLEX_STEP"] if variant == "complex_step" else []
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-Wall", "-Werror", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", *extra,
           "-I", ORACLE, os.path.join(ORACLE, "sanitize_main.c"), os.path.join(ORACLE, "hlbm_oracle.c"),
           "-lm", "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "sanitized oracle run: ok" in r.stdout
