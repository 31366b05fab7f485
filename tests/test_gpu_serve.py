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


def test_device_error_fails_only_its_launch():
    """A launch whose look-back times out (forced from the host: the first
    tile withholds its status word, tiny spin limit) completes with an error
    for its own requests only; requests served before and after are exact."""
    from paper_2106_06161_amd import binding as B

    ex = HipExecutor(streams=2, rounds=24, pool_items=1 << 22)
    srv = ShuffleServer(ex, budget_bytes=256 << 20, small_items=1 << 10, max_inflight=4)
    # the fused kernel (the form with a look-back) for every request
    assert B.bs_probe_set_staged_policy(0) == B.BS_OK
    try:
        first = srv.run(make_requests(20, 100_000, 1_000_000, qps=1e4, seed=3))
        assert len(first.ok()) == 20
        assert B.bs_probe_set_watchdog(2000, 1) == B.BS_OK
        bad = srv.run(make_requests(3, 500_000, 1_000_000, qps=1e4, seed=4))
        torch.cuda.synchronize()
    finally:
        B.bs_probe_set_watchdog(0, 0)
        B.bs_probe_set_staged_policy(2)
    assert bad.completions and not bad.ok()
    assert all("BS_ETIMEOUT" in c.error for c in bad.completions)
    rs = make_requests(20, 100_000, 1_000_000, qps=1e4, seed=5)
    served = {}
    after = srv.run(rs, on_result=lambda r, out: served.__setitem__(r.id, out.clone()))
    torch.cuda.synchronize()
    assert len(after.ok()) == 20 and ex.check_errors() == 0
    for r in rs[:5]:
        want = oracle.shuffle(ex.input_of(r).cpu().numpy(), r.seed, 24)
        assert np.array_equal(served[r.id].cpu().numpy(), want), r


def test_budget_from_free_device_memory():
    ex = HipExecutor(streams=2, rounds=24, pool_items=1 << 20)
    srv = ShuffleServer(ex, small_items=1 << 16)
    rep = srv.run(make_requests(50, 1000, 500_000, qps=1e5, seed=9))
    free, _ = torch.cuda.mem_get_info()
    assert len(rep.ok()) == 50
    assert 0 < rep.budget_bytes <= free + torch.cuda.memory_reserved()
