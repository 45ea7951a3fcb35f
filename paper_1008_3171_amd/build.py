"""Compile the HIP library (libpibbp.so) in-tree for gfx950.

Run as ``python -m paper_1008_3171_amd.build``; __graft_entry__.build() calls
``build()``. The library is always rebuilt when asked, so a stale .so never
survives an explicit build.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpibbp.so")
SOURCES = ["kernels.hip", "abi.cpp", "server.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",
    # packed fp32 instructions stay off (none are wanted in integer code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


PROBE_SRC = os.path.join(PKG, "probe", "valu_rates.hip")
PROBE_BIN = os.path.join(PKG, "probe", "valu_rates")


def build_probe(verbose: bool = False) -> str:
    """The VALU issue-rate probe (a standalone program, not part of the library)."""
    tmp = PROBE_BIN + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", tmp, PROBE_SRC]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr)
    os.replace(tmp, PROBE_BIN)
    return PROBE_BIN


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + [
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-o", tmp,
    ] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns about the device-only target feature; drop that
    err = "\n".join(l for l in res.stderr.splitlines()
                    if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
