"""The server on the GPU: every request's result, produced in the mix of
coalesced launches on several streams, equals the same shuffle run alone and
(for small requests) the oracle, byte for byte."""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd.serve import HipExecutor, ShuffleServer, make_requests

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_the_mix():
    ex = HipExecutor(streams=4, rounds=24, pool_items=1 << 24)
    srv = ShuffleServer(ex, budget_bytes=256 << 20, small_items=1 << 16, max_inflight=8)
    rs = make_requests(400, 100, 2_000_000, qps=2e4, seed=7)
    served = {}
    rep = srv.run(rs, on_result=lambda r, out: served.__setitem__(r.id, out.clone()))
    torch.cuda.synchronize()
    assert len(rep.ok()) == len(rs), [c.error for c in rep.completions if c.error][:3]
    assert rep.batched_launches > 0
    assert ex.check_errors() == 0
    for r in rs:
        x = ex.input_of(r)
        alone = bs.shuffle(x, r.seed, 24)
        assert torch.equal(alone, served[r.id]), r
        if r.n <= 200_000:
            want = oracle.shuffle(x.cpu().numpy(), r.seed, 24)
            assert np.array_equal(served[r.id].cpu().numpy(), want), r
    s = rep.summary()
    assert s["latency_p99_ms"] >= s["latency_p50_ms"] > 0
