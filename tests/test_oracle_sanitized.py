"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

tests/oracle_sanitize.c calls every oracle entry point at the edges of its
arguments. Built once with the sanitizers (any out-of-bounds access, leak,
overflow of a signed value or oversized shift aborts the run) and once
without, it must run clean and print the same results: nothing the oracle
computes depends on undefined behaviour.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def build(tmp_path, name, flags):
    exe = str(tmp_path / name)
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-pthread", "-I", ORACLE] + flags + \
          [os.path.join(HERE, "oracle_sanitize.c"), os.path.join(ORACLE, "pio.c"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_sanitizers_and_matches_the_plain_build(tmp_path):
    plain = build(tmp_path, "plain", ["-O2"])
    san = build(tmp_path, "san", ["-O1", "-g", "-fno-omit-frame-pointer",
                                  "-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    # verify_asan_link_order=0: the environment may preload a library of its own
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    want = subprocess.run([plain], check=True, capture_output=True, text=True, timeout=300)
    got = subprocess.run([san], capture_output=True, text=True, timeout=600, env=env)
    assert got.returncode == 0, got.stderr[-4000:]
    assert "runtime error" not in got.stderr, got.stderr[-4000:]
    assert got.stdout == want.stdout
    lines = want.stdout.splitlines()
    assert len(lines) > 2000
    kinds = {l.split()[0] for l in lines}
    assert kinds == {"pow", "term", "slice", "extract", "certify", "machin"}
