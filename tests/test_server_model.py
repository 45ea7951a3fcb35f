"""The continuous-batching server's bookkeeping, on the CPU.

tests/server_model.cpp runs server.cpp and abi.cpp unchanged on a stand-in
HIP runtime in host memory (tests/fake_hip.cpp), with kernel stand-ins that
count instead of compute. Stream work (copies and kernels) is deferred until
the host waits for it, as on a device, so a buffer rewritten by the host
before queued work has read it, or a result read before its wait, shows up. Seeded streams of queries (both formulas, 1 to
1088 bits, so fused and per-limb-class launches) go through servers with
small steps, a growing slot pool, a device-memory budget below the pool and
one slot, in both pipeline modes. It checks that every head index of every
query is launched exactly once, chunk tables are numbered without gaps,
chunk counters start cleared, counters survive the pool's growth, admission
stays within capacity, and every query comes back once, under its own tag,
with its own head count. Queries withdrawn mid-stream (pi_server_cancel)
never come back, and the same queries submitted again come back right. A
memory budget cut below what is admitted stops admission until the active
queries fit, and loses nothing. The
other front ends get the same checks on 300
whole queries: pi_extract_ex, pi_extract_noalloc, pi_extract_batch (also two
batches issued back to back) and a batch plan launched three times. Built with AddressSanitizer and
UndefinedBehaviorSanitizer.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1008_3171_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


pytestmark = pytest.mark.skipif(
    shutil.which("g++") is None or
    not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
    reason="needs g++ and the HIP headers")


def build(tmp_path, name, flags):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-parameter"] + \
          flags + [os.path.join(HERE, "server_model.cpp"), os.path.join(HERE, "fake_hip.cpp"),
                   os.path.join(CSRC, "abi.cpp"), os.path.join(CSRC, "server.cpp"), "-pthread",
                   "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_server_bookkeeping_on_a_stand_in_runtime(tmp_path):
    san = build(tmp_path, "san", ["-O1", "-g", "-fno-omit-frame-pointer",
                                  "-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    plain = build(tmp_path, "plain", ["-O2"])
    # verify_asan_link_order=0: the environment may preload a library of its own
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([san], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    # the plain build reuses freed memory at once, where the sanitizer's
    # allocator holds it back: the same results either way
    fast = subprocess.run([plain], capture_output=True, text=True, timeout=600)
    assert fast.returncode == 0, fast.stderr[-4000:]
    assert fast.stdout == res.stdout
    lines = res.stdout.splitlines()
    assert len(lines) == 14, res.stdout
    assert lines[0] == "front ends: 300 queries"
    want = {"small steps": 200, "pool growth": 1200, "memory limit": 500, "one at a time": 40,
            "cancel and resubmit": 300}
    streams = [l for l in lines if "withdrawn" in l]
    assert len(streams) == 10, res.stdout
    for l in streams:
        name = l.split(":", 1)[0]
        m = re.search(r"(\d+) queries back, (\d+) withdrawn", l)
        assert m and int(m.group(1)) == want[name], l
        assert (int(m.group(2)) > 0) == (name == "cancel and resubmit"), l
    shrink = [l for l in lines if l.startswith("shrinking budget")]
    assert len(shrink) == 2 and all("120 queries back" in l for l in shrink), res.stdout
    assert lines[-1].endswith("failures 0")
