"""The library's host code (argument checks, the planner, batch planning,
tuning, the server's set-up) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

tests/host_sanitize.cpp links abi.cpp and server.cpp, built with g++ for the
host only, with stand-ins for the kernel launchers. On a host without a GPU
every entry point runs its checks and planning and stops at its first device
call. Built once with the sanitizers and once without, the program must run
clean and print the same results.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1008_3171_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(tmp_path, name, flags):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-parameter"] + \
          flags + [os.path.join(HERE, "host_sanitize.cpp"), os.path.join(CSRC, "abi.cpp"),
                   os.path.join(CSRC, "server.cpp"), "-L", os.path.join(ROCM, "lib"),
                   "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64", "-pthread",
                   "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.mark.skipif(shutil.which("g++") is None or
                    not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="needs g++ and the HIP headers")
def test_host_code_runs_clean_under_sanitizers_and_matches_the_plain_build(tmp_path):
    plain = build(tmp_path, "plain", ["-O2"])
    san = build(tmp_path, "san", ["-O1", "-g", "-fno-omit-frame-pointer",
                                  "-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    # no GPU for this process even where one exists: the program expects none
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    want = subprocess.run([plain], capture_output=True, text=True, timeout=300, env=env)
    assert want.returncode == 0, want.stderr[-4000:]
    # leaks are not checked: the HIP runtime keeps allocations of its own
    # until exit. verify_asan_link_order=0: the environment may preload a
    # library of its own.
    env.update(ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    got = subprocess.run([san], capture_output=True, text=True, timeout=600, env=env)
    assert got.returncode == 0, got.stderr[-4000:]
    assert "runtime error" not in got.stderr, got.stderr[-4000:]
    assert got.stdout == want.stdout
    lines = want.stdout.splitlines()
    kinds = {l.split()[0] for l in lines}
    assert {"plan", "seg", "workspace", "batch_create", "extract_ex", "sum_slice", "combine",
            "tuning", "server_create", "launches"} <= kinds
    # plans were made (not only rejected), and nothing was launched but the
    # combine calls that passed their checks
    assert sum(1 for l in lines if l.startswith("plan") and l.endswith(" 0 " + l.split()[-1])) > 200
