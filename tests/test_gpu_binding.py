"""The binding refuses caller buffers the kernels could write out of bounds
(host tensors, wrong element types, non-contiguous views, short buffers)
before anything reaches the library, and accepts the right ones."""
import pytest
import torch

import paper_1008_3171_amd as pb

pytestmark = pytest.mark.gpu


def test_bad_output_buffers_are_refused():
    P = 320
    good = torch.zeros(pb.limbs(P), dtype=torch.int64, device="cuda")
    status = torch.zeros(4, dtype=torch.int32, device="cuda")
    bad = [
        torch.zeros(pb.limbs(P), dtype=torch.int64),                       # host memory
        torch.zeros(pb.limbs(P), dtype=torch.int32, device="cuda"),        # element type
        torch.zeros(pb.limbs(P) - 1, dtype=torch.int64, device="cuda"),    # one limb short
        torch.zeros(2 * pb.limbs(P), dtype=torch.int64, device="cuda")[::2],  # strided
    ]
    for out in bad:
        with pytest.raises(ValueError):
            pb.extract(pb.BELLARD, 1000, 256, P, out=out, status=status)
        with pytest.raises(ValueError):
            pb.sum_slice(pb.term_id(pb.BELLARD, 0), 1000, 0, 10, P, out=out)
    with pytest.raises(ValueError):
        pb.extract(pb.BELLARD, 1000, 256, P, out=good,
                   status=torch.zeros(3, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        pb.extract(pb.BELLARD, 1000, 256, P, out=good,
                   status=torch.zeros(4, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        pb.combine(torch.zeros(2 * pb.limbs(P) - 1, dtype=torch.int64, device="cuda"), 2, P,
                   256, 7, 100)
    qarr, total = pb.make_queries([(pb.BELLARD, 1000, 64, 128), (pb.BBP, 2000, 256, 320)])
    with pytest.raises(ValueError):
        pb.extract_batch(qarr, 2, torch.zeros(total - 1, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        pb.extract_batch(qarr, 3, torch.zeros(total, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        pb.BatchPlan(qarr, 2, torch.zeros(total, dtype=torch.int64, device="cuda"),
                     torch.zeros(7, dtype=torch.int32, device="cuda"))
    # the right buffers still work
    out, st = pb.extract(pb.BELLARD, 1000, 256, P, out=good, status=status)
    torch.cuda.synchronize()
    assert pb.status_of(st)[0] == pb.PI_OK
