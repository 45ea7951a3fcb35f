"""Static view of the library's gfx950 code: registers and innermost loops.

Compiles ``csrc/kernels.hip`` for the device only, to assembly, with the
library's own flags, and reports for a kernel its register and scratch use
(from the code object's metadata) and every innermost loop (a backward branch
whose range holds no other backward branch) with its instruction mix. The
ladder's window loops show the cost of a squaring directly: six fp64
instructions (two multiplies, two FMAs, a round and an add) in the binary64
classes, and the multiply-adds of a Montgomery step in the integer classes.

    python -m paper_1008_3171_amd.isa --kernel "head_kernel_args<5>"
"""
from __future__ import annotations

import argparse
import collections
import os
import re
import shutil
import subprocess
import tempfile

from . import build as _build

KERNELS_SRC = os.path.join(_build.CSRC, "kernels.hip")


def device_asm(path: str | None = None) -> str:
    """Assembly text of kernels.hip for gfx950 (device code only)."""
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared", "-fPIC", "-fvisibility=hidden")]
    with tempfile.TemporaryDirectory() as tmp:
        out = path or os.path.join(tmp, "kernels.s")
        cmd = [_build.hipcc()] + flags + ["--offload-device-only", "-S",
                                           "-I", os.path.join(_build.ROOT, "include"),
                                           "-I", _build.CSRC, "-o", out, KERNELS_SRC]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + res.stderr)
        with open(out) as f:
            return f.read()


def demangle(names):
    names = list(names)
    tool = shutil.which("c++filt")
    if not tool or not names:
        return {n: n for n in names}
    res = subprocess.run([tool], input="\n".join(names), capture_output=True, text=True)
    out = res.stdout.splitlines()
    if res.returncode != 0 or len(out) != len(names):
        return {n: n for n in names}
    return dict(zip(names, out))


def functions(asm: str) -> dict:
    """Kernel symbol -> (instructions, {label: index of the next instruction})."""
    lines = asm.splitlines()
    found = {}
    i = 0
    while i < len(lines):
        m = re.match(r"^([A-Za-z_][\w.$]*):", lines[i].split(";")[0].strip())
        if m and i > 0 and "@function" in "".join(lines[max(0, i - 3):i]):
            name = m.group(1)
            insts, labels = [], {}
            j = i + 1
            while j < len(lines) and not lines[j].startswith(".Lfunc_end"):
                s = lines[j].split(";")[0].strip()
                lm = re.match(r"^(\.L\w+):", s)
                if lm:
                    labels[lm.group(1)] = len(insts)
                elif s and not s.startswith("."):
                    insts.append(s)
                j += 1
            found[name] = (insts, labels)
            i = j
        i += 1
    return found


def metadata(asm: str) -> dict:
    """Kernel symbol -> {key: value} from the code object's metadata."""
    m = re.search(r"\.amdgpu_metadata(.*?)\.end_amdgpu_metadata", asm, re.S)
    if not m:
        return {}
    out, cur = {}, None
    for line in m.group(1).splitlines():
        if re.match(r"^  - \.", line):
            cur = {}
        km = re.match(r"^  [ -] \.(\w+):\s+(\S+)\s*$", line)
        if cur is not None and km:
            cur[km.group(1)] = km.group(2)
            if km.group(1) == "name":
                out[km.group(2)] = cur
    return out


def innermost_loops(insts, labels):
    """(first, last) instruction index of every innermost loop."""
    loops = []
    for i, s in enumerate(insts):
        m = re.match(r"^s_(?:cbranch_\w+|branch)\s+(\.L\w+)", s)
        if m and labels.get(m.group(1), len(insts)) <= i:
            loops.append((labels[m.group(1)], i))
    return sorted(l for l in loops
                  if not any(o != l and l[0] <= o[0] and o[1] <= l[1] for o in loops))


def mix(insts, first, last):
    return collections.Counter(insts[k].split()[0] for k in range(first, last + 1))


def find(asm: str, kernel: str):
    """The symbol whose demangled name starts with `kernel` (e.g.
    "pibbp::head_kernel_args<5>" or "head_kernel_args<5>")."""
    funcs = functions(asm)
    names = demangle(funcs)
    want = kernel if "::" in kernel else "pibbp::" + kernel
    hits = [s for s, d in names.items() if re.sub(r"^void ", "", d).startswith(want + "(")]
    if len(hits) != 1:
        raise KeyError("%s: %d matches" % (kernel, len(hits)))
    return hits[0], funcs[hits[0]]


def report(asm: str, kernel: str) -> str:
    sym, (insts, labels) = find(asm, kernel)
    md = metadata(asm).get(sym, {})
    rows = ["%s: %d instructions; VGPRs %s, SGPRs %s, spills %s/%s, LDS %s B, scratch %s B" % (
        kernel, len(insts), md.get("vgpr_count"), md.get("sgpr_count"),
        md.get("vgpr_spill_count"), md.get("sgpr_spill_count"),
        md.get("group_segment_fixed_size"), md.get("private_segment_fixed_size"))]
    for a, b in innermost_loops(insts, labels):
        c = mix(insts, a, b)
        valu = sum(v for k, v in c.items() if k.startswith("v_"))
        salu = sum(v for k, v in c.items() if k.startswith("s_"))
        ops = ", ".join("%s %d" % kv for kv in sorted(c.items(), key=lambda kv: (-kv[1], kv[0]))
                        if kv[0].startswith("v_"))
        rows.append("  loop at %d: %d VALU, %d SALU/branch: %s" % (a, valu, salu, ops))
    return "\n".join(rows)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--kernel", action="append",
                    help="demangled name without arguments; repeatable (default: the "
                         "single-query head kernel at 5 limbs and the fused head kernel)")
    ap.add_argument("--asm", help="also write the assembly here")
    args = ap.parse_args(argv)
    asm = device_asm(args.asm)
    for k in args.kernel or ["head_kernel_args<5>", "head_kernel_fused"]:
        print(report(asm, k))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
