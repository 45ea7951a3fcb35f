"""Static checks of the library's gfx950 code (CPU: hipcc cross-compiles).

The device code is compiled to assembly with the library's own flags and
checked for what the design relies on:
* no packed fp32 arithmetic anywhere;
* the head kernels neither spill nor use scratch, and the single-query head
  kernel at 5 limbs fits seven workgroups of 256 lanes per CU (72 VGPRs);
* a binary64 squaring is six fp64 instructions (two multiplies, two FMAs, a
  round, an add) in every window loop of the ladder: 2-, 3- and 4-bit windows
  add the digit's extraction and ldexp, five-bit windows add their separate
  digit step (multiply, round, FMA and the extraction and ldexp);
* a step on 31-bit digits (R = 2^62) is nine 32-bit multiplies;
* bench.py's per-term instruction model prices every modulus class's window
  and the carry step as they were compiled.
"""
import collections
import shutil

import pytest

from paper_1008_3171_amd import build as pbuild
from paper_1008_3171_amd import isa

pytestmark = pytest.mark.skipif(shutil.which(pbuild.hipcc()) is None, reason="needs hipcc")

HEAD_KERNELS = ["head_kernel_args<%d>" % L for L in (1, 2, 3, 4, 5, 6, 8, 12, 17)] + \
               ["head_kernel_ptr<%d>" % L for L in (1, 2, 3, 4, 5, 6, 8, 12, 17)] + \
               ["head_kernel_fused"]


@pytest.fixture(scope="module")
def asm():
    return isa.device_asm()


def loops_of(asm, kernel):
    _, (insts, labels) = isa.find(asm, kernel)
    return [isa.mix(insts, a, b) for a, b in isa.innermost_loops(insts, labels)]


def valu(c):
    return collections.Counter({k: v for k, v in c.items() if k.startswith("v_")})


def window(squarings, digit_step):
    """The VALU mix of one binary64 window loop."""
    c = collections.Counter({"v_mul_f64": 2 * squarings, "v_fma_f64": 2 * squarings,
                             "v_rndne_f64_e32": squarings, "v_add_f64": squarings,
                             "v_bfe_u32": 1, "v_ldexp_f64": 1})
    if digit_step:
        c.update({"v_mul_f64": 1, "v_fma_f64": 1, "v_rndne_f64_e32": 1})
    return c


def test_no_packed_fp32_arithmetic(asm):
    for op in ("v_pk_add_f32", "v_pk_mul_f32", "v_pk_fma_f32"):
        assert op not in asm, op


def test_head_kernels_keep_everything_in_registers(asm):
    md = isa.metadata(asm)
    for k in HEAD_KERNELS:
        sym, _ = isa.find(asm, k)
        m = md[sym]
        assert m["vgpr_spill_count"] == "0" and m["sgpr_spill_count"] == "0", k
        assert m["private_segment_fixed_size"] == "0", k
    sym, _ = isa.find(asm, "head_kernel_args<5>")
    assert int(md[sym]["vgpr_count"]) <= 72          # 7 x 4 waves of 256 lanes per CU
    assert 7 * int(md[sym]["group_segment_fixed_size"]) <= 160 * 1024


@pytest.mark.parametrize("kernel", ["head_kernel_args<5>", "head_kernel_ptr<5>",
                                    "head_kernel_fused"])
def test_binary64_squaring_is_six_instructions(asm, kernel):
    found = [valu(c) for c in loops_of(asm, kernel)]
    for bits in (2, 3, 4):
        assert window(bits, False) in found, (kernel, bits)
    assert window(5, True) in found, kernel
    # every loop that squares in binary64 is one of these windows (the fused
    # kernel may add one register move)
    for c in found:
        if c["v_rndne_f64_e32"] and c["v_bfe_u32"]:
            s = c["v_add_f64"]
            want = window(s, c["v_rndne_f64_e32"] == s + 1)
            extra = c - want
            assert not (want - c) and sum(extra.values()) <= 1, (kernel, c)


def test_montgomery_step_on_31_bit_digits_is_nine_multiplies(asm):
    for kernel in ("head_kernel_args<5>", "head_kernel_fused"):
        muls = [c["v_mad_u64_u32"] + c["v_mul_lo_u32"] for c in loops_of(asm, kernel)
                if c["v_mad_u64_u32"] >= 7]
        assert muls and all(m == 9 for m in muls), (kernel, muls)


def test_per_term_model_matches_the_compiled_window_loops(asm):
    # bench.py prices each modulus class at (window bits W) x (per squaring)
    # + (per window) instructions per whole window; the compiled head kernel
    # has a window loop of exactly that many VALU instructions for each class
    # (class 62 steps one bit at a time; one copy of its loop keeps one more
    # mask). The carry step over the digit sums is 28 at 5 limbs.
    import bench
    counts = {}
    for c in loops_of(asm, "head_kernel_args<5>"):
        v = sum(valu(c).values())
        counts[v] = counts.get(v, 0) + 1
    for name, _, W, per_sq, per_win, _, _ in bench.KERNEL_CLASSES:
        want = W * per_sq + per_win
        assert counts.get(want, 0) >= 1, (name, want, counts)
    assert counts.get(16) and counts.get(17)
    assert round(bench.FP_EXTRA_PER_TERM * 120 - 81 * 120 / 256) == 28
    carry = [c for c in loops_of(asm, "head_kernel_args<5>")
             if valu(c) == collections.Counter({"v_ldexp_f64": 7, "v_floor_f64_e32": 7,
                                                "v_fmac_f64_e32": 7, "v_add_f64": 7,
                                                "v_mov_b64_e32": 1})]
    assert len(carry) == 4                         # one per binary64 class
