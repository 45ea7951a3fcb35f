"""CPU-side checks of the C-ABI library: it loads, exports every function
include/pibbp.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

import oracle
import paper_1008_3171_amd as pb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pibbp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*PI_API\s+(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pi_[a-z_0-9]+)\s*\(",
                                 src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = pb.load()
    names = declared_functions()
    assert {"pi_extract", "pi_extract_ex", "pi_sum_slice", "pi_extract_batch",
            "pi_workspace_size", "pi_strerror", "pi_server_create", "pi_server_step"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_strerror():
    lib = pb.load()
    for code in (0, 1, -1, -2, -3, -4, -5, 99):
        assert lib.pi_strerror(code)


@pytest.mark.parametrize("formula", [pb.BBP, pb.BELLARD])
def test_head_term_count_matches_oracle_tables(formula):
    rows, step, _ = oracle.series_table(formula)
    for n in (1, 2, 7, 9, 100, 10 ** 6, 10 ** 10 + 1, 10 ** 12, 2 * 10 ** 15 - 3):
        d = n - 1
        want = sum(max(0, (d + c) // step + 1) for _, c, _, _ in rows)
        assert pb.head_terms(formula, n) == want
    if formula == pb.BELLARD:
        assert pb.head_terms(formula, 10 ** 6) == 700001


def test_invalid_arguments_are_rejected_synchronously():
    lib = pb.load()
    dummy = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    null = ctypes.c_void_p(0)
    E = -1
    assert lib.pi_extract_ex(2, 10, 8, 72, dummy, null, null) == E          # formula
    assert lib.pi_extract_ex(1, 0, 8, 72, dummy, null, null) == E           # n = 0
    assert lib.pi_extract_ex(1, 10, 0, 72, dummy, null, null) == E          # nbits = 0
    assert lib.pi_extract_ex(1, 10, 80, 72, dummy, null, null) == E         # P < nbits
    assert lib.pi_extract_ex(1, 10, 8, 2000, dummy, null, null) == E        # P > max
    assert lib.pi_extract_ex(1, 10, 8, 72, null, null, null) == E           # out = NULL
    assert lib.pi_sum_slice(pb.term_id(1, 7), 10, 0, 5, 64, dummy, null) == E
    assert lib.pi_sum_slice(pb.term_id(0, 4), 10, 0, 5, 64, dummy, null) == E
    assert lib.pi_sum_slice(pb.term_id(1, 0), 10, 6, 5, 64, dummy, null) == E  # k0 > k1
    assert lib.pi_extract(1, 10, 0, dummy, null) == E
    # the static-scratch variant validates the same way, before any device call
    lib.pi_extract_noalloc.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
    assert lib.pi_extract_noalloc(2, 10, 8, 72, dummy, null, null) == E
    assert lib.pi_extract_noalloc(1, 0, 8, 72, dummy, null, null) == E
    assert lib.pi_extract_noalloc(1, 10, 8, 2000, dummy, null, null) == E
    assert lib.pi_extract_noalloc(1, 10, 8, 72, null, null, null) == E
    assert lib.pi_extract_noalloc(1, 2 ** 61, 8, 72, dummy, null, null) == -4
    # moduli from 2^54 up are outside the supported range
    assert lib.pi_extract_ex(1, 2 ** 61, 8, 72, dummy, null, null) == -4
    assert lib.pi_extract_ex(1, 2 ** 55, 8, 72, dummy, null, null) == -4


def test_arith_mode_roundtrip_and_limits():
    lib = pb.load()
    assert pb.get_arith() == pb.ARITH_FAST
    pb.set_arith(pb.ARITH_INTEGER)
    assert pb.get_arith() == pb.ARITH_INTEGER
    pb.set_arith(pb.ARITH_FAST)
    assert pb.get_arith() == pb.ARITH_FAST
    assert lib.pi_set_arith(2) == -1 and lib.pi_set_arith(-1) == -1
    assert pb.get_arith() == pb.ARITH_FAST


def test_arith_mode_belongs_to_the_calling_thread():
    import threading
    lib = pb.load()
    seen = {}

    def other():
        seen["start"] = lib.pi_get_arith()
        lib.pi_set_arith(pb.ARITH_INTEGER)
        seen["set"] = lib.pi_get_arith()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen == {"start": pb.ARITH_FAST, "set": pb.ARITH_INTEGER}
    assert pb.get_arith() == pb.ARITH_FAST          # this thread's mode is untouched
    # and the planner follows the calling thread's mode: class 31 and the
    # R = 2^62 class from 2^31 exist only in integer mode
    pb.set_arith(pb.ARITH_INTEGER)
    try:
        cls_int = {s["cls"] for s in pb.plan_head(pb.BELLARD, 10 ** 10, 320)}
    finally:
        pb.set_arith(pb.ARITH_FAST)
    cls_fast = {s["cls"] for s in pb.plan_head(pb.BELLARD, 10 ** 10, 320)}
    assert 31 in cls_int and 31 not in cls_fast


def test_tuning_roundtrip_and_limits():
    lib = pb.load()
    before = pb.get_tuning(5)
    pb.set_tuning(5, 6, 32)
    assert pb.get_tuning(5) == (6, 32)
    pb.set_tuning(5, *before)
    assert pb.get_tuning(5) == before
    # a limb count maps to its kernel instance: 7 limbs run on the 8-limb one
    before8 = pb.get_tuning(8)
    pb.set_tuning(7, 3, 48)
    assert pb.get_tuning(8) == (3, 48) and pb.get_tuning(7) == (3, 48)
    pb.set_tuning(8, *before8)
    assert lib.pi_set_tuning(5, 0, 0) == -1          # run cap 0
    assert lib.pi_set_tuning(18, 0, 64) == -1        # no such limb count
    assert lib.pi_set_tuning(-2, 0, 64) == -1
    assert lib.pi_set_tuning(5, 65, 64) == -1
    # the fused launch of batches and serving steps has a shape of its own
    before_f = pb.get_tuning(pb.TUNE_FUSED)
    before5 = pb.get_tuning(5)
    pb.set_tuning(pb.TUNE_FUSED, 5, 1024)
    assert pb.get_tuning(pb.TUNE_FUSED) == (5, 1024) and pb.get_tuning(5) == before5
    pb.set_tuning(pb.TUNE_FUSED, *before_f)
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    assert lib.pi_get_tuning(0, ctypes.byref(a), ctypes.byref(b)) == -1


def test_binding_fails_loudly_without_a_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError, match="no GPU"):
        pb.extract(pb.BELLARD, 1000, 256)


def test_binding_refuses_host_buffers_before_the_library(monkeypatch):
    # every wrapper that takes a caller's buffer checks it first: host tensors
    # never reach the kernels. Nothing here reaches the library, so the test
    # runs without a GPU once the binding's device check is told there is one.
    torch = pytest.importorskip("torch")
    monkeypatch.setattr(torch.cuda, "is_available", lambda: True)
    P = 320
    host = torch.zeros(pb.limbs(P), dtype=torch.int64)
    hst = torch.zeros(4, dtype=torch.int32)
    with pytest.raises(ValueError, match="GPU"):
        pb.extract(pb.BELLARD, 1000, 256, P, out=host, status=hst)
    with pytest.raises(ValueError, match="GPU"):
        pb.extract_noalloc(pb.BELLARD, 1000, 256, P, host, hst)
    with pytest.raises(ValueError, match="GPU"):
        pb.extract_default(pb.BELLARD, 1000, 256, out=host)
    with pytest.raises(ValueError, match="GPU"):
        pb.sum_slice(pb.term_id(pb.BELLARD, 0), 1000, 0, 10, P, out=host)
    with pytest.raises(ValueError, match="GPU"):
        pb.combine(torch.zeros(2 * pb.limbs(P), dtype=torch.int64), 2, P, 256, 7, 100,
                   out=host, status=hst)
    qarr, total = pb.make_queries([(pb.BELLARD, 1000, 64, 128), (pb.BBP, 2000, 256, 320)])
    with pytest.raises(ValueError, match="GPU"):
        pb.extract_batch(qarr, 2, torch.zeros(total, dtype=torch.int64), status=False)
    with pytest.raises(ValueError, match="GPU"):
        pb.BatchPlan(qarr, 2, torch.zeros(total, dtype=torch.int64))
    with pytest.raises(ValueError, match="outside"):
        pb.extract_batch(qarr, 3, host, status=False)
