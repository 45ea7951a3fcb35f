"""pi_extract_noalloc (static device scratch, nothing allocated) gives
exactly what pi_extract_ex gives, through the C ABI. The static-scratch
calls run back to back on one stream, sharing the scratch: a large query,
then a smaller one (fewer limbs, smaller n), then the most limbs the scratch
serves, then the abstract's worked example."""
import ctypes

import pytest
import torch

import paper_1008_3171_amd as pb

pytestmark = pytest.mark.gpu

CASES = [(pb.BELLARD, 10 ** 10, 256, 320),       # 5 limbs, 7.0e9 head terms
         (pb.BBP, 123_457, 64, 96),              # 2 limbs, a smaller query
         (pb.BELLARD, 10 ** 8 + 1, 1000, 1088),  # 17 limbs, 35 scratch words
         (pb.BELLARD, 9, 8, 72)]                 # bits 9..16 are 0x3F


def launch(fn, f, n, w, P, stream):
    lib = pb.load()
    out = torch.full((pb.limbs(P),), -1, dtype=torch.int64, device="cuda")
    st = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    entry = getattr(lib, fn)
    entry.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    entry.restype = ctypes.c_int
    rc = entry(f, n, w, P, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.data_ptr()),
               ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, (fn, rc)
    return out, st


def test_noalloc_equals_extract_ex_on_consecutive_calls():
    stream = torch.cuda.current_stream()
    want = [launch("pi_extract_ex", *c, stream) for c in CASES]
    torch.cuda.synchronize()
    got = [launch("pi_extract_noalloc", *c, stream) for c in CASES]   # no wait between
    torch.cuda.synchronize()
    for c, (wo, ws), (go, gs) in zip(CASES, want, got):
        assert torch.equal(go, wo) and torch.equal(gs, ws), c
        assert pb.status_of(gs)[0] == pb.PI_OK, c
    out, st = got[-1]
    assert pb.to_int(out, 72) >> 64 == 0x3F
