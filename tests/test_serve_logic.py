"""Scheduling logic of the shuffle server on the CPU.

The executor here is a test double (the oracle behind the server's Executor
interface, with a fake clock); the product executor is HipExecutor.  These
tests cover admission by budget, FIFO order, coalescing, failure isolation,
requests too large for the budget, and cancellation.
"""
import numpy as np
import pytest

import oracle
from paper_2106_06161_amd.serve import Request, ShuffleServer, make_requests


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        self.t += 1e-6
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Computes each launch with the oracle; a launch completes after
    `polls_to_finish` polls.  Inputs are slices of a seeded pool per element
    size, assigned in placement order like the GPU executor does."""

    def __init__(self, polls_to_finish=3, fail_poll_ids=(), fail_launch_ids=(), fail_result_ids=(),
                 free=1 << 30):
        rng = np.random.default_rng(0)
        self.pools = {4: rng.integers(0, 2**32, size=1 << 20, dtype=np.uint32),
                      8: rng.integers(0, 2**63, size=1 << 20, dtype=np.int64).view(np.uint64)}
        self.cursor = {4: 0, 8: 0}
        self.where = {}
        self.polls_to_finish = polls_to_finish
        self.fail_poll_ids = set(fail_poll_ids)
        self.fail_launch_ids = set(fail_launch_ids)
        self.fail_result_ids = set(fail_result_ids)
        self.free = free
        self.launches = []
        self.lanes = []
        self.live = 0
        self.max_live = 0

    def place(self, r):
        eb = r.elem_bytes
        if self.cursor[eb] + r.n > len(self.pools[eb]):
            self.cursor[eb] = 0
        self.where[r.id] = (eb, self.cursor[eb])
        self.cursor[eb] += r.n

    def input_of(self, r):
        eb, first = self.where[r.id]
        return self.pools[eb][first:first + r.n]

    def launch(self, reqs, lane=1):
        self.lanes.append(lane)
        if any(r.id in self.fail_launch_ids for r in reqs):
            raise RuntimeError("launch failed")
        self.launches.append([r.id for r in reqs])
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return {"reqs": reqs, "polls": 0}

    def poll(self, h):
        h["polls"] += 1
        if any(r.id in self.fail_poll_ids for r in h["reqs"]):
            raise RuntimeError("device fault in this launch")
        return h["polls"] >= self.polls_to_finish

    def results(self, h):
        # a launch that finished but reported a device-side status (the GPU
        # executor's per-launch error word) raises here, like HipExecutor
        if any(r.id in self.fail_result_ids for r in h["reqs"]):
            raise RuntimeError("BS_ETIMEOUT: device-side error in this launch")
        return {r.id: oracle.shuffle(self.input_of(r), r.seed, 24) for r in h["reqs"]}

    def free_bytes(self):
        return self.free

    def release(self, h):
        self.live -= 1


def server(ex, budget, clock=None, **kw):
    clock = clock or FakeClock()
    return ShuffleServer(ex, budget, clock=clock.now, sleep=clock.sleep, **kw)


def reqs(sizes, dtypes=None, gap=1e-4):
    dtypes = dtypes or ["uint32"] * len(sizes)
    return [Request(i, i * gap, n, d, 1000 + i) for i, (n, d) in enumerate(zip(sizes, dtypes))]


def test_every_request_completes_with_its_own_result():
    ex = FakeExecutor()
    rs = make_requests(200, 10, 5000, qps=5e4, seed=1)
    got = {}
    rep = server(ex, 1 << 30, small_items=1000).run(rs, on_result=lambda r, out: got.__setitem__(r.id, out))
    assert len(rep.ok()) == 200
    for r in rs:
        assert np.array_equal(got[r.id], oracle.shuffle(ex.input_of(r), r.seed, 24))


def test_budget_is_never_exceeded_and_admission_is_fifo():
    ex = FakeExecutor(polls_to_finish=5)
    rs = reqs([300, 500, 200, 800, 100, 700, 400], gap=0.0)
    budget = 4 * 1000  # bytes: at most ~1000 uint32 records reserved at once
    rep = server(ex, budget, small_items=0).run(rs)
    assert len(rep.ok()) == len(rs)
    assert rep.max_reserved_bytes <= budget
    admitted = [c.admitted for c in sorted(rep.completions, key=lambda c: c.request.id)]
    assert admitted == sorted(admitted)


def test_small_requests_coalesce_per_element_size():
    ex = FakeExecutor(polls_to_finish=50)
    sizes = [10, 20, 5000, 30, 40, 6000, 50]
    dtypes = ["uint32", "int64", "uint32", "float32", "int64", "int64", "uint32"]
    rs = reqs(sizes, dtypes, gap=0.0)
    rep = server(ex, 1 << 30, small_items=1000).run(rs)
    assert len(rep.ok()) == len(rs)
    groups = sorted(sorted(g) for g in ex.launches)
    # big requests alone; small uint32/float32 (4-byte) together; small int64 together
    assert groups == sorted([[2], [5], [0, 3, 6], [1, 4]])
    assert rep.batched_launches == 2


def test_batch_limits_split_groups():
    ex = FakeExecutor(polls_to_finish=50)
    rs = reqs([100] * 10, gap=0.0)
    server(ex, 1 << 30, small_items=1000, max_batch_requests=4).run(rs)
    assert sorted(len(g) for g in ex.launches) == [2, 4, 4]


def test_failed_launch_fails_only_its_requests():
    ex = FakeExecutor(fail_poll_ids={3})
    rs = reqs([2000, 2000, 2000, 2000, 2000])
    rep = server(ex, 1 << 30, small_items=1000).run(rs)
    failed = {c.request.id for c in rep.completions if c.error}
    assert failed == {3}
    assert len(rep.ok()) == 4
    ex2 = FakeExecutor(fail_launch_ids={1})
    rep2 = server(ex2, 1 << 30, small_items=1000).run(reqs([2000, 2000, 2000]))
    assert {c.request.id for c in rep2.completions if c.error} == {1}


def test_device_error_fails_its_launch_and_hands_out_nothing():
    """A launch whose device status is set after it finished (e.g. a look-back
    that timed out) fails all of its requests and only those; on_result is
    never called for them."""
    ex = FakeExecutor(fail_result_ids={2, 7})
    rs = reqs([2000, 2000, 2000, 10, 20, 30, 2000, 40, 50], gap=0.0)
    got = {}
    rep = server(ex, 1 << 30, small_items=1000).run(rs, on_result=lambda r, out: got.__setitem__(r.id, out))
    failed = {c.request.id for c in rep.completions if c.error}
    want = set().union(*(set(g) for g in ex.launches if {2, 7} & set(g)))
    assert {2, 7} <= want and want != set(range(len(rs)))
    assert failed == want
    assert set(got) == set(range(len(rs))) - want
    assert len(rep.ok()) == len(rs) - len(want)


def test_budget_defaults_to_the_executors_free_memory():
    ex = FakeExecutor(polls_to_finish=5, free=4 * 1000)
    rs = reqs([300, 500, 200, 800, 100, 700, 400], gap=0.0)
    rep = server(ex, None, small_items=0).run(rs)
    assert rep.budget_bytes == 4000 and rep.max_reserved_bytes <= 4000
    assert len(rep.ok()) == len(rs)
    ex.free = 10  # every request now exceeds the budget, read again at the start of the run
    rep = server(ex, None, small_items=0).run(rs)
    assert not rep.ok()


def test_request_larger_than_budget_is_rejected_alone():
    ex = FakeExecutor()
    rs = reqs([100, 10_000, 100])
    rep = server(ex, 4 * 1000, small_items=0).run(rs)
    errs = {c.request.id: c.error for c in rep.completions}
    assert errs[1] and "budget" in errs[1]
    assert errs[0] is None and errs[2] is None


def test_cancelled_request_is_skipped():
    ex = FakeExecutor()
    rs = reqs([100, 100, 100], gap=1.0)
    srv = server(ex, 1 << 30, small_items=0)
    srv.cancel(1)
    rep = srv.run(rs)
    assert sorted(c.request.id for c in rep.completions) == [0, 2]


def test_inflight_limit():
    ex = FakeExecutor(polls_to_finish=20)
    rs = reqs([2000] * 12, gap=0.0)
    server(ex, 1 << 30, small_items=1000, max_inflight=3).run(rs)
    assert ex.max_live <= 3


def test_request_stream_recipe():
    rs = make_requests(5000, 1000, 100_000_000, qps=100.0, seed=5)
    n = np.array([r.n for r in rs])
    assert n.min() >= 1000 and n.max() < 100_000_000
    # log-uniform: the median is near sqrt(lo * hi)
    assert 2e5 < np.median(n) < 6e5
    gaps = np.diff([r.arrival for r in rs])
    assert abs(gaps.mean() - 0.01) < 0.001
    assert {r.dtype for r in rs} == {"uint32", "int64", "float32"}


class _InstantExecutor:
    """Launches finish at their second poll; no data is moved."""

    def __init__(self):
        self.k = 0

    def place(self, r):
        pass

    def launch(self, reqs, lane=1):
        self.k += 1
        return [self.k, 0]

    def poll(self, h):
        h[1] += 1
        return h[1] > 1

    def results(self, h):
        return {}

    def release(self, h):
        pass


def test_scheduler_cost_is_linear_in_requests():
    """Host-side scheduling of a closed-loop burst (every request arrives at
    once) must stay O(1) per request: 50,000 requests in well under a second
    per 10,000 on this container."""
    import time

    reqs = make_requests(50_000, 1000, 100_000_000, 1e12, 5)
    t0 = time.perf_counter()
    rep = ShuffleServer(_InstantExecutor(), 32 << 30).run(reqs)
    dt = time.perf_counter() - t0
    s = rep.summary()
    assert s["completed"] == 50_000 and s["failed"] == 0
    assert dt < 10.0, dt


def test_size_policy_launches_small_groups_first_then_shortest():
    ex = FakeExecutor(polls_to_finish=3)
    sizes = [9000, 3000, 50, 7000, 60, 5000]
    rs = reqs(sizes, gap=0.0)
    server(ex, 1 << 30, small_items=1000, max_inflight=2, small_slots=1, policy="size", max_wait=1e9).run(rs)
    # one slot for large requests: the small group first, then large ones by size
    assert ex.launches[0] == [2, 4] and ex.lanes[0] == 0
    big = [g[0] for g in ex.launches[1:]]
    assert big == [1, 5, 3, 0] and all(lane == 1 for lane in ex.lanes[1:])


def test_size_policy_ages_out_long_waits():
    ex = FakeExecutor(polls_to_finish=400)
    # request 0 (largest) arrives first; with max_wait 0 it is launched first
    rs = reqs([9000, 3000, 5000], gap=0.0)
    server(ex, 1 << 30, small_items=1000, max_inflight=2, small_slots=1, policy="size", max_wait=0.0).run(rs)
    assert [g[0] for g in ex.launches] == [0, 1, 2]


def test_fifo_policy_keeps_admission_order():
    ex = FakeExecutor(polls_to_finish=3)
    rs = reqs([9000, 3000, 7000, 5000], gap=0.0)
    server(ex, 1 << 30, small_items=1000, max_inflight=1, policy="fifo").run(rs)
    assert [g[0] for g in ex.launches] == [0, 1, 2, 3]
    assert set(ex.lanes) == {1}


def test_small_slots_keep_room_for_small_groups():
    ex = FakeExecutor(polls_to_finish=50)
    rs = reqs([5000] * 8 + [10, 20], gap=0.0)
    srv = server(ex, 1 << 30, small_items=1000, max_inflight=4, small_slots=2, policy="size")
    rep = srv.run(rs)
    assert len(rep.ok()) == 10
    # the small group was launched while large requests were still waiting
    first_small = next(i for i, g in enumerate(ex.launches) if g == [8, 9])
    assert first_small < 8
