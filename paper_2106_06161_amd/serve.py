"""Continuous-batching shuffle server (single GPU).

Requests (size n, payload dtype, 64-bit seed, arrival time) are served in
real time:

  admission   a request is admitted once it has arrived and its output
              bytes fit the HBM budget (by default the device's free memory
              at the start of the run, less a reserve; FIFO: a request that
              does not fit holds back the ones behind it);
  coalescing  admitted requests of at most `small_items` records are grouped
              by element size into one bs_shuffle_batched launch (their inputs
              sit back to back in a device-resident pool); larger requests get
              a bs_shuffle launch of their own;
  overlap     launches go to several HIP streams (policy "size", the
              default: small groups on a stream of their own, large
              requests shortest first on the others, none waiting longer
              than max_wait; policy "fifo": admission order, round-robin),
              so requests that arrive while others run are admitted as
              memory frees up and their work overlaps on the device;
  completion  an event per launch; a request's latency is the time from its
              scheduled arrival to the moment its launch is seen complete.

Every request's result depends only on its own input bytes, n, dtype size,
seed and the round count: grouping, stream and timing never change a byte.

The executor owns all device work (HipExecutor); the scheduling logic only
talks to the Executor interface below.
"""
from __future__ import annotations

import dataclasses
import gc
import heapq
import math
import sys
import time
from collections import deque
from typing import Callable, Protocol

import numpy as np

ELEM_BYTES = {"uint32": 4, "float32": 4, "int64": 8}


@dataclasses.dataclass
class Request:
    id: int
    arrival: float  # seconds after the start of the run
    n: int
    dtype: str
    seed: int

    @property
    def elem_bytes(self) -> int:
        return ELEM_BYTES[self.dtype]

    @property
    def out_bytes(self) -> int:
        return self.n * self.elem_bytes


@dataclasses.dataclass
class Completion:
    request: Request
    admitted: float
    done: float
    batch_size: int
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.request.arrival


class Executor(Protocol):
    """Device side of the server.  A launch covers one or more requests of
    one element size; `poll` returns True once its results are final."""

    def place(self, req: Request) -> None: ...
    def launch(self, reqs: list[Request], lane: int = 1) -> object: ...  # lane 0: small groups, 1: large
    def poll(self, handle: object) -> bool: ...
    def results(self, handle: object) -> dict[int, object]: ...  # raises if the launch failed on the device
    def release(self, handle: object) -> None: ...
    def free_bytes(self) -> int: ...  # device memory the server may reserve for outputs


@dataclasses.dataclass
class ServeReport:
    completions: list[Completion]
    wall_s: float
    launches: int
    batched_launches: int
    max_reserved_bytes: int
    budget_bytes: int

    def ok(self) -> list[Completion]:
        return [c for c in self.completions if c.error is None]

    def summary(self) -> dict:
        ok = self.ok()
        lat = np.array([c.latency for c in ok]) if ok else np.zeros(1)
        items = sum(c.request.n for c in ok)
        return {
            "requests": len(self.completions),
            "completed": len(ok),
            "failed": len(self.completions) - len(ok),
            "wall_s": self.wall_s,
            "requests_per_s": len(ok) / self.wall_s if self.wall_s > 0 else math.nan,
            "Gelem_per_s": items / self.wall_s / 1e9 if self.wall_s > 0 else math.nan,
            "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
            "latency_p90_ms": float(np.percentile(lat, 90) * 1e3),
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
            "latency_max_ms": float(lat.max() * 1e3),
            **self._by_size(ok),
            "launches": self.launches,
            "batched_launches": self.batched_launches,
            "mean_requests_per_launch": len(self.completions) / max(self.launches, 1),
            "max_reserved_bytes": self.max_reserved_bytes,
            "budget_bytes": self.budget_bytes,
        }


    @staticmethod
    def _by_size(ok: list[Completion]) -> dict:
        """p50 / p99 latency of requests up to 10^6 records and above."""
        out = {}
        for name, sel in (("le_1e6", lambda n: n <= 1_000_000), ("gt_1e6", lambda n: n > 1_000_000)):
            lat = np.array([c.latency for c in ok if sel(c.request.n)])
            if lat.size:
                out[f"latency_p50_{name}_ms"] = float(np.percentile(lat, 50) * 1e3)
                out[f"latency_p99_{name}_ms"] = float(np.percentile(lat, 99) * 1e3)
        return out


class _Grouper:
    """Admitted requests on their way to launches: a request above small_items
    is a launch of its own; smaller ones are coalesced per element size, in
    admission order, up to max_requests requests and max_items records per
    launch.  flush() closes the open small groups.

    Launch order.  policy "fifo": closed launches in the order they closed.
    policy "size": closed small-request groups first (in order), then single
    large requests shortest first, except that a large request admitted at
    least max_wait seconds ago goes first, so none starves.  O(log n) per
    request (heap and queue entries of launched requests are dropped lazily)."""

    def __init__(self, small_items: int, max_requests: int, max_items: int, policy: str = "size",
                 max_wait: float = 0.05):
        if policy not in ("fifo", "size"):
            raise ValueError(f"unknown launch policy {policy!r}")
        self.small_items, self.max_requests, self.max_items = small_items, max_requests, max_items
        self.policy, self.max_wait = policy, max_wait
        self.ready: deque[list[Request]] = deque()  # fifo: every closed launch; size: small groups
        self.big: dict[int, Request] = {}  # size: large requests not launched yet, by sequence number
        self.by_size: list[tuple[int, int]] = []  # size: heap of (records, seq)
        self.by_age: deque[tuple[float, int]] = deque()  # size: (admitted, seq) in admission order
        self.seq = 0
        self.open: dict[int, list[Request]] = {}
        self.open_items: dict[int, int] = {}

    def add(self, r: Request, now: float = 0.0) -> None:
        if r.n > self.small_items:
            if self.policy == "fifo":
                self.ready.append([r])
            else:
                self.big[self.seq] = r
                heapq.heappush(self.by_size, (r.n, self.seq))
                self.by_age.append((now, self.seq))
                self.seq += 1
            return
        eb = r.elem_bytes
        cur = self.open.setdefault(eb, [])
        if cur and (len(cur) >= self.max_requests or self.open_items[eb] + r.n > self.max_items):
            self.ready.append(cur)
            cur = self.open[eb] = []
            self.open_items[eb] = 0
        cur.append(r)
        self.open_items[eb] = self.open_items.get(eb, 0) + r.n

    def flush(self) -> None:
        for cur in self.open.values():
            if cur:
                self.ready.append(cur)
        self.open.clear()
        self.open_items.clear()

    def pop(self, now: float = 0.0, allow_big: bool = True) -> list[Request] | None:
        """The next closed launch, or None (allow_big=False: small groups only)."""
        if self.ready:
            return self.ready.popleft()
        if not allow_big or not self.big:
            return None
        while self.by_age[0][1] not in self.big:
            self.by_age.popleft()
        if now - self.by_age[0][0] >= self.max_wait:
            return [self.big.pop(self.by_age.popleft()[1])]
        while True:
            _, seq = heapq.heappop(self.by_size)
            if seq in self.big:
                return [self.big.pop(seq)]

    def has_closed(self) -> bool:
        return bool(self.ready) or bool(self.big)

    def __bool__(self) -> bool:
        return bool(self.ready) or bool(self.big) or any(self.open.values())


class ShuffleServer:
    """budget_bytes: output bytes the admitted, unfinished requests may hold
    at once; None takes the executor's free device memory at the start of
    each run (free_bytes())."""

    def __init__(self, executor: Executor, budget_bytes: int | None = None, small_items: int = 1 << 20,
                 max_batch_requests: int = 2048, max_batch_items: int = 1 << 26, max_inflight: int = 16,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 policy: str = "size", max_wait: float = 0.05, small_slots: int = 2):
        self.ex = executor
        self.fixed_budget = None if budget_bytes is None else int(budget_bytes)
        self.budget = self.fixed_budget if self.fixed_budget is not None else 0
        self.small_items = small_items
        self.max_batch_requests = max_batch_requests
        self.max_batch_items = max_batch_items
        self.max_inflight = max_inflight
        self.policy = policy
        self.max_wait = max_wait
        # "size": launch slots large requests may not take, kept for small groups
        self.small_slots = min(small_slots, max_inflight - 1) if policy == "size" else 0
        self.clock = clock
        self.sleep = sleep
        self.cancelled: set[int] = set()

    def cancel(self, request_id: int) -> None:
        """Drop a request that has not been admitted yet."""
        self.cancelled.add(request_id)

    def run(self, requests: list[Request], on_result: Callable[[Request, object], None] | None = None) -> ServeReport:
        # no cyclic-GC pauses inside the scheduling loop (the request objects
        # hold no cycles; reference counting still frees them)
        gc_enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, on_result)
        finally:
            if gc_enabled:
                gc.enable()

    def _run(self, requests: list[Request], on_result: Callable[[Request, object], None] | None) -> ServeReport:
        self.budget = self.fixed_budget if self.fixed_budget is not None else int(self.ex.free_bytes())
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        grouper = _Grouper(self.small_items, self.max_batch_requests, self.max_batch_items, self.policy,
                           self.max_wait)
        admit_time: dict[int, float] = {}
        inflight: list[tuple[object, list[Request]]] = []
        completions: list[Completion] = []
        reserved = max_reserved = 0
        launches = batched = 0
        t0 = self.clock()
        while pending or grouper or inflight:
            now = self.clock() - t0
            # retire finished launches
            still = []
            for handle, reqs in inflight:
                try:
                    finished = self.ex.poll(handle)
                except Exception as exc:  # a failed launch fails only its own requests
                    finished, err = True, f"{type(exc).__name__}: {exc}"
                else:
                    err = None
                if not finished:
                    still.append((handle, reqs))
                    continue
                t_done = self.clock() - t0
                outs = {}
                if err is None:
                    try:
                        outs = self.ex.results(handle)
                    except Exception as exc:
                        err = f"{type(exc).__name__}: {exc}"
                for r in reqs:
                    completions.append(Completion(r, admit_time[r.id], t_done, len(reqs), err))
                    if err is None and on_result is not None:
                        on_result(r, outs[r.id])
                    reserved -= r.out_bytes
                self.ex.release(handle)
            inflight = still
            # admit arrived requests while the budget allows (FIFO)
            while pending and pending[0].arrival <= now:
                r = pending[0]
                if r.id in self.cancelled:
                    pending.popleft()
                    continue
                if r.out_bytes > self.budget:
                    pending.popleft()
                    completions.append(Completion(r, now, now, 0, "request exceeds the HBM budget"))
                    continue
                if reserved + r.out_bytes > self.budget:
                    break
                pending.popleft()
                reserved += r.out_bytes
                max_reserved = max(max_reserved, reserved)
                admit_time[r.id] = now
                try:
                    self.ex.place(r)
                except Exception as exc:
                    reserved -= r.out_bytes
                    completions.append(Completion(r, now, self.clock() - t0, 0, f"{type(exc).__name__}: {exc}"))
                    continue
                grouper.add(r, now)
            # launch what is admitted, as slots allow; open small groups are
            # closed only when a slot is free for them
            while grouper and len(inflight) < self.max_inflight:
                # "size": small requests go out as soon as a slot is free;
                # "fifo": open groups close only when nothing else is ready
                if self.policy == "size" or not grouper.has_closed():
                    grouper.flush()
                big_ok = len(inflight) < self.max_inflight - self.small_slots
                g = grouper.pop(self.clock() - t0, allow_big=big_ok)
                if g is None:
                    break
                small = len(g) > 1 or g[0].n <= self.small_items
                try:
                    handle = self.ex.launch(g, lane=0 if (small and self.policy == "size") else 1)
                except Exception as exc:
                    t_fail = self.clock() - t0
                    for r in g:
                        completions.append(Completion(r, admit_time[r.id], t_fail, len(g),
                                                      f"{type(exc).__name__}: {exc}"))
                        reserved -= r.out_bytes
                    continue
                inflight.append((handle, g))
                launches += 1
                batched += len(g) > 1
            if not inflight and not grouper and pending:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(min(wait, 0.001))
            elif inflight:
                self.sleep(0)
        wall = self.clock() - t0
        return ServeReport(completions, wall, launches, batched, max_reserved, self.budget)


# ------------------------------------------------------------ HIP executor --
class HipExecutor:
    """Runs launches with libbshuffle on one GPU.

    Inputs live in device-resident pools (one per element size) filled once
    with seeded random bytes; a request's input is the next `n` records of
    its pool, assigned in admission order, so consecutive small requests of
    one element size are contiguous and one bs_shuffle_batched covers them.
    Outputs are allocated per launch and returned as views.

    Each stream has its own workspace.  After every launch the stream
    moves that workspace's device-side error word into a pinned host slot
    (bs_workspace_error_async); results() raises for a launch whose slot is
    not BS_OK (a look-back that timed out, a malformed batch), so the server
    fails exactly that launch's requests and hands out none of its bytes.
    """

    def __init__(self, device="cuda:0", streams: int = 4, rounds: int = 24, pool_items: int = 1 << 27,
                 pool_seed: int = 2106, batch_items: int = 1 << 26, batch_requests: int = 2048,
                 reserve_bytes: int = 4 << 30):
        import torch

        import paper_2106_06161_amd as bs

        self.torch, self.bs = torch, bs
        self.device = torch.device(device)
        self.rounds = rounds
        self.reserve_bytes = reserve_bytes
        self.streams = [torch.cuda.Stream(self.device) for _ in range(streams)]
        self.next_stream = 0
        # room for the staged form of the largest request of either element
        # size (bs_shuffle takes it where the tuned table prefers it) and for
        # the largest coalesced batch
        ws_bytes = max(bs.workspace_bytes(pool_items, elem_bytes=4, staged=True),
                       bs.workspace_bytes(pool_items, elem_bytes=8, staged=True),
                       bs.workspace_bytes(batch_items, batch_requests))
        self.workspaces = [bs.make_workspace(ws_bytes, device=self.device, stream=s) for s in self.streams]
        self.status = torch.full((4096,), -1, dtype=torch.int32).pin_memory()
        self.next_slot = 0
        gen = torch.Generator(device=self.device)
        gen.manual_seed(pool_seed)
        self.pools = {
            4: torch.randint(-2**31, 2**31 - 1, (pool_items,), dtype=torch.int32, device=self.device, generator=gen),
            8: torch.randint(-2**63, 2**63 - 1, (pool_items,), dtype=torch.int64, device=self.device, generator=gen),
        }
        self.cursor = {4: 0, 8: 0}
        self.where: dict[int, tuple[int, int]] = {}  # request id -> (elem_bytes, first record in its pool)
        torch.cuda.synchronize(self.device)

    def place(self, req: Request) -> None:
        eb = req.elem_bytes
        pool = self.pools[eb]
        if req.n > pool.numel():
            raise ValueError(f"request of {req.n} records exceeds the input pool")
        if self.cursor[eb] + req.n > pool.numel():
            self.cursor[eb] = 0
        self.where[req.id] = (eb, self.cursor[eb])
        self.cursor[eb] += req.n

    def input_of(self, req: Request):
        eb, first = self.where[req.id]
        return self.pools[eb][first:first + req.n]

    def launch(self, reqs: list[Request], lane: int = 1):
        torch, bs = self.torch, self.bs
        # lane 0 (coalesced small requests) has the first stream to itself, so
        # small launches never queue behind a large one; large launches take
        # the other streams in turn
        if lane == 0 or len(self.streams) == 1:
            si = 0
        else:
            si = 1 + self.next_stream % (len(self.streams) - 1)
            self.next_stream += 1
        stream, ws = self.streams[si], self.workspaces[si]
        slot = self.next_slot
        self.next_slot = (slot + 1) % self.status.numel()
        self.status[slot] = -1
        eb = reqs[0].elem_bytes
        firsts = [self.where[r.id][1] for r in reqs]
        contiguous = all(firsts[i] + reqs[i].n == firsts[i + 1] for i in range(len(reqs) - 1))
        with torch.cuda.stream(stream):
            if len(reqs) == 1:
                x = self.input_of(reqs[0])
                y = bs.shuffle(x, reqs[0].seed, self.rounds, workspace=ws)
                outs = {reqs[0].id: y}
                keep = ()
            elif contiguous:
                total = sum(r.n for r in reqs)
                x = self.pools[eb][firsts[0]:firsts[0] + total]
                offs = np.zeros(len(reqs) + 1, dtype=np.int64)
                np.cumsum([r.n for r in reqs], out=offs[1:])
                seeds = np.array([r.seed & (2**64 - 1) for r in reqs], dtype=np.uint64).view(np.int64)
                off_h = torch.from_numpy(offs).pin_memory()
                sd_h = torch.from_numpy(seeds).pin_memory()
                off_d = off_h.to(self.device, non_blocking=True)
                sd_d = sd_h.to(self.device, non_blocking=True)
                y = bs.shuffle_batched(x, off_d, sd_d, self.rounds, workspace=ws)
                outs = {r.id: y[int(offs[i]):int(offs[i + 1])] for i, r in enumerate(reqs)}
                keep = (off_h, sd_h, off_d, sd_d)
            else:  # a pool wrap split the run: fall back to one launch per request
                outs = {r.id: bs.shuffle(self.input_of(r), r.seed, self.rounds, workspace=ws) for r in reqs}
                keep = ()
            bs.workspace_error_async(ws, self.status[slot:slot + 1], stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return {"event": ev, "outs": outs, "keep": keep, "stream": stream, "slot": slot}

    def poll(self, handle) -> bool:
        return handle["event"].query()

    def results(self, handle) -> dict[int, object]:
        st = int(self.status[handle["slot"]])
        if st != 0:
            raise self.bs.BShuffleError(st, "device-side error in this launch")
        return handle["outs"]

    def free_bytes(self) -> int:
        """Free device memory (plus what torch's allocator holds unused), less
        a reserve for workspaces and the allocator's own rounding."""
        torch = self.torch
        free, _ = torch.cuda.mem_get_info(self.device)
        cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        return max(0, int(free + cached - self.reserve_bytes))

    def release(self, handle) -> None:
        handle["outs"] = None
        handle["keep"] = None

    def check_errors(self) -> int:
        for s, ws in zip(self.streams, self.workspaces):
            err = self.bs.workspace_error(ws, stream=s)
            if err:
                return err
        return 0


def make_requests(count: int, lo: int, hi: int, qps: float, seed: int) -> list[Request]:
    """Poisson arrivals at `qps`, log-uniform sizes in [lo, hi], dtype uniform
    over uint32 / int64 / float32, 64-bit seeds (PCG64(seed))."""
    from .workloads import request_stream

    return [Request(d["id"], d["arrival"], d["n"], d["dtype"], d["seed"])
            for d in request_stream(count, lo, hi, qps, seed)]


def main(argv=None) -> int:
    import argparse
    import json

    p = argparse.ArgumentParser(description="Run the shuffle server on a synthetic request stream.")
    p.add_argument("--requests", type=int, default=2000)
    p.add_argument("--lo", type=int, default=1000)
    p.add_argument("--hi", type=int, default=100_000_000)
    p.add_argument("--qps", type=float, default=0.0,
                   help="0: measure closed-loop capacity C first, then run at each of --loads x C")
    p.add_argument("--loads", default="0.8", help="comma-separated fractions of C (with --qps 0)")
    p.add_argument("--budget-gib", type=float, default=0.0,
                   help="output budget; 0: the device's free memory at the start of each run")
    p.add_argument("--streams", type=int, default=4)
    p.add_argument("--rounds", type=int, default=24)
    p.add_argument("--seed", type=int, default=5)
    p.add_argument("--policy", choices=("size", "fifo"), default="size")
    p.add_argument("--max-inflight", type=int, default=16)
    p.add_argument("--small-slots", type=int, default=2)
    a = p.parse_args(argv)
    ex = HipExecutor(streams=a.streams, rounds=a.rounds)
    budget = int(a.budget_gib * 2**30) if a.budget_gib > 0 else None
    server = ShuffleServer(ex, budget, policy=a.policy, max_inflight=a.max_inflight,
                           small_slots=a.small_slots)
    out = {"requests": a.requests, "policy": a.policy, "max_inflight": a.max_inflight,
           "small_slots": a.small_slots, "streams": a.streams}
    if a.qps > 0:
        rates = [a.qps]
    else:
        cap = server.run(make_requests(a.requests, a.lo, a.hi, 1e12, a.seed)).summary()
        out["closed_loop"] = cap
        print(f"closed loop: {cap['requests_per_s']:.1f} requests/s", file=sys.stderr, flush=True)
        rates = [float(f) * cap["requests_per_s"] for f in a.loads.split(",")]
    out["open_loop"] = []
    for qps in rates:
        rep = server.run(make_requests(a.requests, a.lo, a.hi, qps, a.seed + 1)).summary()
        out["open_loop"].append(dict(rep, qps=qps))
        print(f"open loop at {qps:.1f} requests/s: p50 {rep['latency_p50_ms']:.2f} ms, "
              f"p99 {rep['latency_p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    out["device_error"] = ex.check_errors()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
