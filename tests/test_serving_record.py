"""The full serving stream's recorded results (records/serving_stream_20000.json,
written on the GPU by `python -m paper_1008_3171_amd.serving stream --record`)
checked against the oracle on the CPU: every query with n <= 10^5 and a
seeded sample of 300 with 10^5 < n <= 10^7, each its P-bit sum, N and
certification. The record's queries must be the seeded stream's."""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
from paper_1008_3171_amd import workloads

RECORD = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "records",
                      "serving_stream_20000.json")


@pytest.mark.skipif(not os.path.exists(RECORD), reason="no serving record")
def test_recorded_serving_results_equal_the_oracle():
    rec = json.load(open(RECORD))
    stream = workloads.serving_stream(rec["queries"], seed=rec["seed"])
    rows = rec["checked_results"]
    assert len(rows) > 4000
    assert rec["identical_to_burst"] and rec["all_certified"]
    for tag, f, n, w, P, S, code, N in rows:
        assert stream[tag][1:] == (f, n, w, P), tag

    def one(row):
        tag, f, n, w, P, S, code, N = row
        want_S, want_N, cert = oracle.extract(f, n, w, P)
        return (int(S, 16), code, N) == (want_S, 0 if cert else 1, want_N)

    with ThreadPoolExecutor(8) as ex:
        ok = list(ex.map(one, rows))
    bad = [rows[i][0] for i, good in enumerate(ok) if not good]
    assert not bad, bad[:10]
