#!/usr/bin/env python3
"""Benchmark of the bijective shuffle on one MI355X.

One step = one bs_shuffle of the headline workload: n = 2^27 + 1 uint32 values
drawn uniform from [0, 2^32) with PCG64(7), seed 7, 24 rounds (the paper's
setting), padded domain 2^28.  That single fused kernel covers every step of
the method: parameters and round keys, the cipher, keep flags and scan with
decoupled look-back, the random gather and the output stores.

Prints ONE JSON line:
  value        Gelem/s over the K timed steps (inputs resident in HBM)
  roofline     the fused kernel against the HBM peak: algorithmic bytes
               (one read + one write of every record, 8 B per uint32 item)
               per launch over the kernel's average duration (HIP events on
               the launch stream), plus the HBM traffic measured by rocprofv3
               when a summary for the current kernel sources is committed
  cpu_baseline the sequential CPU oracle on a bounded sample (one thread)
  ceilings     measured device copy and random-gather rates, the cipher+scan
               kernel alone, the 4-round and power-of-two variants
  fusion       the fused kernel against the less-fused forms of Sec. 6
               (Bijective0: cipher table, compaction, gather as three passes;
               Bijective1: a separate tile-count and scan pass before the
               gather), the LCG bijection in the same fused kernel, and the
               permutation-output and un-shuffle variants
  small        n = 100,000 uint32, 4 rounds: per-call latency
  large        n = 10^9 uint32 and 2.5e8 records of 16 bytes, 24 rounds
  batched      4,096 independent shuffles in one launch vs 4,096 calls
  serving      the continuous-batching server: capacity, p50 / p99 latency

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
N_HEADLINE = (1 << 27) + 1
SEED = 7
ROUNDS = 24
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_shuffle_u32_n2p27p1.txt")
# device code of the fused kernel: the committed traffic figures hold while
# these files and the launch shape are unchanged
KERNEL_SOURCES = [
    "paper_2106_06161_amd/csrc/shuffle_impl.h",
    "paper_2106_06161_amd/csrc/tile_scan.h",
    "paper_2106_06161_amd/csrc/vphilox_round.h",
    "paper_2106_06161_amd/csrc/kernels.h",
    "paper_2106_06161_amd/csrc/staged.hip",
]
# the staged form's passes at the headline (k = 28, even); the first pass
# takes its two-workgroups-per-CU shape once rounds x 5 >= 80
STAGED_KERNELS = ["bsd::(anonymous namespace)::staged_zero_kernel(bsd::StagedArgs)",
                  "void bsd::(anonymous namespace)::staged_first_kernel<4, false, {small}>(bsd::StagedArgs)",
                  "void bsd::(anonymous namespace)::staged_second_kernel<4>(bsd::StagedArgs)",
                  "bsd::(anonymous namespace)::staged_scan_kernel(bsd::StagedArgs)",
                  "void bsd::(anonymous namespace)::staged_place_kernel<4>(bsd::StagedArgs)"]
DEPTH_STAGED = 16


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_label(launch: dict, rounds: int = ROUNDS) -> str:
    """The kernels that run the headline step (even k, 32-bit indices): the
    staged form's passes, or the fused kernel."""
    if launch["depth"] == DEPTH_STAGED:
        small = "true" if rounds * 5 >= 80 else "false"
        return " + ".join(k.format(small=small) for k in STAGED_KERNELS)
    if launch["depth"] in (8, 9):  # kept images compacted through LDS (9: pipelined cipher)
        pipe = "true" if launch["depth"] == 9 else "false"
        return "bsd::shuffle_compact_kernel<4, false, {waves}, {items}, ".format(**launch) + pipe + ", 0, true, false>"
    return "bsd::shuffle_single_kernel<4, false, {waves}, {items}, {depth}, false, 0, true, 0>".format(**launch)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse_args():
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--rounds", type=int, default=ROUNDS)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-ceilings", action="store_true")
    p.add_argument("--no-fusion", action="store_true")
    p.add_argument("--fusion-sweep", action="store_true",
                   help="also time every fusion form over n = 2^20 .. 2^29 (+1)")
    p.add_argument("--no-large", action="store_true")
    p.add_argument("--no-sweep", action="store_true",
                   help="skip the size sweep (fused kernel beside the same-footprint random-read ceiling over "
                        "n = 2^w, 2^w+1, w = 8..30, u32 and u64)")
    p.add_argument("--gather-sweep", action="store_true",
                   help="add a random gather with an index array to every sweep point")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-serving", action="store_true")
    p.add_argument("--serve-requests", type=int, default=100_000)
    p.add_argument("--serve-loads", default="0.5,0.8", help="open-loop rates as fractions of the closed-loop capacity")
    p.add_argument("--profile-footprint", action="store_true",
                   help="profiler run: a copy of known size, then the random-read probe over every footprint and "
                        "record size; no extras")
    p.add_argument("--profile-staged", action="store_true",
                   help="profiler run: a copy of known size, then --steps staged shuffles of the headline workload "
                        "(and of n = 10^9 uint32 with --staged-large); no extras")
    p.add_argument("--staged-large", action="store_true")
    p.add_argument("--profile-unshuffle", action="store_true",
                   help="profiler run: --steps staged un-shuffles (bs_unshuffle_staged) of the headline workload's "
                        "shuffled output; no extras")
    p.add_argument("--profile-large", action="store_true",
                   help="profiler run: a copy of known size, then the large workloads (10^9 uint32, 2.5e8 x 16 B) "
                        "and the u64 n = 2^27+1 shuffle, --steps each; no extras")
    p.add_argument("--profile", action="store_true",
                   help="profiler run: one copy of known size, then the steps; no extras")
    p.add_argument("--profile-small", action="store_true",
                   help="profiler run of the small workload (n = 100,000 uint32, 4 rounds): eager calls, graph "
                        "replays, the launch floor and the round-trip probe; no extras")
    p.add_argument("--profile-batched", action="store_true",
                   help="profiler run of the batched workload: --steps batched launches, no extras")
    p.add_argument("--traffic-record", nargs="+", metavar="PATH",
                   help="CPU only: print the headline kernel's traffic record (the file the roofline's "
                        "traffic comes from) from rocprofv3 output: KT_DIR FETCH_DIR WRITE_DIR BENCH_JSON "
                        "[SQ_DIR [TCC_DIR]] (kernel trace, FETCH_SIZE, WRITE_SIZE, the --profile run's JSON line, "
                        "SQ and TCC counter runs of bench.py --profile)")
    return p.parse_args()


class Timer:
    """HIP events on one stream (torch's current stream, where the library launches)."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def run(self, fn, iters: int, warm: int = 2) -> float:
        torch = self.torch
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(iters)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(iters)]
        for i in range(iters):
            starts[i].record(self.stream)
            fn()
            ends[i].record(self.stream)
        torch.cuda.synchronize()
        return sum(s.elapsed_time(e) for s, e in zip(starts, ends)) / iters * 1e-3


def committed_traffic(digest: str, launch: dict, rounds: int = ROUNDS):
    """The committed traffic record when it was taken on the same kernel
    sources, launch shape and round count (the record is of the 24-round
    headline), else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.loads(fh.read())
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_digest") != digest or rec.get("launch") != launch or rounds != ROUNDS:
        return None
    return rec


def traffic_record(paths: list) -> dict:
    """The headline kernel's HBM traffic per launch from rocprofv3 CSVs of
    `bench.py --profile` runs: FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the same counter reads for the run's first kernel, a
    copy of known size; the kernel's average duration from the kernel trace;
    optional SQ and TCC counters.  The launch shape comes from the profiled
    run's JSON line."""
    import csv
    import glob

    if not 4 <= len(paths) <= 6:
        raise SystemExit("--traffic-record needs KT_DIR FETCH_DIR WRITE_DIR BENCH_JSON [SQ_DIR [TCC_DIR]]")
    kt, fetch_dir, write_dir, bench_json = paths[:4]
    sq = paths[4] if len(paths) > 4 else None
    tcc = paths[5] if len(paths) > 5 else None
    copy_bytes = ((N_HEADLINE * 4) // 16) * 16

    def is_main(name):
        return "shuffle_compact_kernel" in name or "shuffle_single_kernel" in name or "::staged_" in name

    def rows(d, pattern):
        with open(glob.glob(os.path.join(d, pattern))[0]) as fh:
            return list(csv.DictReader(fh))

    # the step's kernels: one fused kernel, or the staged form's passes (each
    # launched once per step); per-kernel averages are summed over the step
    main_rows = [r for r in rows(kt, "*kernel_stats.csv") if is_main(r["Name"])]
    if not main_rows:
        raise SystemExit("no shuffle kernel in the trace")
    calls = {int(r["Calls"]) for r in main_rows}
    if len(calls) != 1:
        raise SystemExit(f"the step's kernels ran different numbers of times: {[(r['Name'], r['Calls']) for r in main_rows]}")

    def counter(d, name):
        rs = rows(d, "*counter_collection.csv")
        copy = [float(r["Counter_Value"]) for r in rs if "copy16_kernel" in r["Kernel_Name"] and r["Counter_Name"] == name]
        per = {}
        for r in rs:
            if is_main(r["Kernel_Name"]) and r["Counter_Name"] == name:
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return copy, per

    def per_step(per):
        return sum(sum(v) / len(v) for v in per.values())

    fc, fk = counter(fetch_dir, "FETCH_SIZE")
    wc, wk = counter(write_dir, "WRITE_SIZE")
    fscale = copy_bytes / (fc[0] * 1024.0)
    wscale = copy_bytes / (wc[0] * 1024.0)
    fetch = per_step(fk) * 1024.0 * fscale
    write = per_step(wk) * 1024.0 * wscale
    with open(bench_json) as fh:
        launch = json.loads(fh.read().strip().splitlines()[-1])["config"]["launch"]
    rec = {
        "kernel": " + ".join(r["Name"] for r in main_rows),
        "workload": "n=2^27+1 uint32, seed 7, 24 rounds, domain 2^28",
        "kernel_source_digest": kernel_source_digest(),
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "hbm_bytes_per_launch": fetch + write,
        "fetch_scale_from_copy": fscale,
        "write_scale_from_copy": wscale,
        "copy_probe_bytes": copy_bytes,
        "copy_fetch_kib": fc[0],
        "copy_write_kib": wc[0],
        "kernel_fetch_kib_avg": per_step(fk),
        "kernel_write_kib_avg": per_step(wk),
        "kernel_avg_ms_rocprof": sum(float(r["AverageNs"]) for r in main_rows) / 1e6,
        "kernel_calls_rocprof": calls.pop(),
        "per_kernel_ms_rocprof": {r["Name"]: float(r["AverageNs"]) / 1e6 for r in main_rows},
        "per_kernel_fetch_bytes": {k: sum(v) / len(v) * 1024.0 * fscale for k, v in fk.items()},
        "per_kernel_write_bytes": {k: sum(v) / len(v) * 1024.0 * wscale for k, v in wk.items()},
        "launch": launch,
    }
    if sq:
        for name in ("SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
                     "SQ_WAVES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"):
            _, v = counter(sq, name)
            if v:
                rec[name.lower() + "_per_launch"] = per_step(v)
    if tcc:
        for name in ("TCC_EA0_RDREQ_sum", "TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_RDREQ_LEVEL_sum",
                     "TCC_EA0_RDREQ_32B_sum", "TCC_BUBBLE_sum"):
            c, v = counter(tcc, name)
            if v:
                rec[name.lower() + "_per_launch"] = per_step(v)
            if c:
                rec[name.lower() + "_copy"] = c[0]
    return rec


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _pinned_trials(fn, trials: int) -> list[float]:
    """Runs fn `trials` times with this thread pinned to one core (restored after)."""
    old = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    if old:
        os.sched_setaffinity(0, {min(old)})
    try:
        times = []
        for _ in range(trials):
            t0 = time.perf_counter()
            fn()
            times.append(time.perf_counter() - t0)
        return times
    finally:
        if old:
            os.sched_setaffinity(0, old)


def cpu_baseline(x, y_gpu, trials: int = 3) -> dict:
    """The oracle, single thread pinned to one core, on the headline's own
    input bytes (n = 2^27+1 uint32, seed 7, 24 rounds): mean of `trials`
    runs.  Its output is compared whole with the GPU's output of the timed
    steps."""
    import numpy as np

    import oracle

    n = x.shape[0]
    first = {}

    def run():
        out = oracle.shuffle(x, SEED, ROUNDS)
        first.setdefault("out", out)

    times = _pinned_trials(run, trials)
    same = bool(np.array_equal(first["out"], y_gpu))
    dt = sum(times) / len(times)
    return {
        "value": n / dt / 1e9,
        "unit": "Gelem/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the headline workload itself: n=2^27+1 uint32 uniform (PCG64 seed 7), seed 7, {ROUNDS} rounds, "
                  f"domain 2^28; mean of {trials} runs ({dt:.2f} s each, min {min(times):.2f} s) pinned to one "
                  f"core of {cpu_model()} ({os.cpu_count()} logical CPUs)",
        "gpu_output_equal": same,
    }


def cpu_std_shuffle(x, trials: int = 3) -> dict:
    """std::shuffle (Fisher-Yates, std::mt19937_64), one thread pinned to one core, same input bytes."""
    import oracle

    n = x.shape[0]
    times = _pinned_trials(lambda: oracle.std_shuffle_u32(x, SEED), trials)
    dt = sum(times) / len(times)
    return {"value": n / dt / 1e9, "unit": "Gelem/s", "cores": 1, "kind": "std::shuffle",
            "sample": f"n=2^27+1 uint32 (the headline's input bytes), std::mt19937_64(7), mean of {trials} runs "
                      f"({dt:.3f} s each) pinned to one core of {cpu_model()}"}


def bench_batched_small(torch, bs, B, W, np, dev, timer, rounds) -> list:
    """Batches of many small segments (the statistical tests' shape: 100,000
    permutations of n = 5, 100 and 1,000, seeds 1..100,000; and 65,536
    segments of 10..10^4 records, PCG64 seed 4): one wavefront per segment of
    at most 1,024 records against every segment in a tile (same bytes)."""
    cases = [(f"100000 x n={n}", np.arange(100_001, dtype=np.int64) * n, np.arange(1, 100_001, dtype=np.uint64))
             for n in (5, 100, 1000)]
    b = W.batch(65536, 10, 10_000, seed=4)
    cases.append(("65536 x [10, 1e4]", b["offsets"], b["seeds"]))
    out = []
    for name, offsets, seeds in cases:
        total, S = int(offsets[-1]), len(offsets) - 1
        x = torch.arange(total, dtype=torch.int64, device=dev).to(torch.int32)
        y = torch.empty_like(x)
        off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(dev)
        sd = torch.from_numpy(np.ascontiguousarray(seeds, dtype=np.uint64).view(np.int64)).to(dev)
        ws = bs.make_workspace(bs.workspace_bytes(total, S), device=dev)
        row = {"workload": name, "records": total}
        ref = None
        try:
            for small, key in ((1, "one_wavefront"), (0, "tiles_only")):
                B._check(B.bs_probe_set_batch_small(small), "bs_probe_set_batch_small")
                t = timer.run(lambda: bs.shuffle_batched(x, off, sd, rounds, out=y, workspace=ws), 5)
                row[key + "_ms"] = t * 1e3
                if ref is None:
                    ref = y.clone()
                elif not torch.equal(y, ref):
                    raise RuntimeError(f"small-segment paths differ on {name}")
        finally:
            B.bs_probe_set_batch_small(1)
        row["Gelem_s"] = total / row["one_wavefront_ms"] / 1e6
        if bs.workspace_error(ws) != 0:
            raise RuntimeError("device-side error in the small-segment batches")
        out.append(row)
        del x, y, ws, ref
    return out


def bench_batched(torch, bs, W, np, dev, stream, timer, rounds) -> dict:
    """4,096 independent shuffles: one batched launch (graph replay) against
    4,096 bs_shuffle calls on one stream, eager and captured in one graph."""
    b = W.batch(4096, 100, 1_000_000, seed=3)
    total, S = b["total"], 4096
    x = torch.arange(total, dtype=torch.int64, device=dev).to(torch.int32)
    y = torch.empty_like(x)
    off = torch.from_numpy(b["offsets"]).to(dev)
    sd = torch.from_numpy(b["seeds"].view(np.int64)).to(dev)
    ws_b = bs.make_workspace(bs.workspace_bytes(total, S), device=dev)
    ws_s = bs.make_workspace(bs.workspace_bytes(int(b["sizes"].max())), device=dev)
    offsets = [int(v) for v in b["offsets"]]
    seeds = [int(v) for v in b["seeds"]]
    views = [(x[offsets[s]:offsets[s + 1]], y[offsets[s]:offsets[s + 1]], seeds[s]) for s in range(S)
             if offsets[s + 1] > offsets[s]]

    def one_batched():
        bs.shuffle_batched(x, off, sd, rounds, out=y, workspace=ws_b)

    def per_call():
        for xs, ys, sdv in views:
            bs.shuffle(xs, sdv, rounds, out=ys, workspace=ws_s)

    def graph_of(fn):
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            fn()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            fn()
        torch.cuda.synchronize()
        return g

    t_batched_eager = timer.run(one_batched, 5)
    g1 = graph_of(one_batched)
    t_batched_graph = timer.run(g1.replay, 5)
    t0 = time.perf_counter()
    per_call()
    torch.cuda.synchronize()
    t_calls_eager = time.perf_counter() - t0
    t_calls_eager = min(t_calls_eager, timer.run(per_call, 2, warm=0))
    gN = graph_of(per_call)
    t_calls_graph = timer.run(gN.replay, 3)
    err = bs.workspace_error(ws_b) or bs.workspace_error(ws_s)
    del g1, gN
    return {
        "workload": "4,096 shuffles, sizes floor(exp(U(ln 100, ln 1e6))) from PCG64(3), uint32 payload, "
                    f"{rounds} rounds, per-segment 64-bit seeds",
        "total_items": total,
        "batched_graph_ms": t_batched_graph * 1e3,
        "batched_eager_ms": t_batched_eager * 1e3,
        "per_call_eager_ms": t_calls_eager * 1e3,
        "per_call_graph_ms": t_calls_graph * 1e3,
        "batched_Gelem_s": total / t_batched_graph / 1e9,
        "per_call_Gelem_s": total / t_calls_eager / 1e9,
        "speedup_vs_per_call_eager": t_calls_eager / t_batched_graph,
        "speedup_vs_per_call_graph": t_calls_graph / t_batched_graph,
        "device_error": int(err),
    }


def bench_fusion(torch, bs, B, W, dev, stream, timer, rounds, n, x=None, y=None) -> dict:
    """One shuffle of n uint32 values in each fusion form; every form's output
    is checked equal to the fused kernel's."""
    sp = stream.cuda_stream
    if x is None:
        x = torch.from_numpy(W.uniform_u32(n, seed=SEED)).to(dev)
        y = torch.empty_like(x)
    # a workspace with no room for the staged form: bs_shuffle runs the fused kernel
    ws = bs.make_workspace(bs.workspace_bytes(n), device=dev)
    ref = torch.empty_like(x)
    scratch = torch.empty(B.bs_probe_unfused_scratch_bytes(n), dtype=torch.uint8, device=dev)

    def fused():
        bs.shuffle(x, SEED, rounds, out=y, workspace=ws)

    def two_pass():
        B._check(B.bs_probe_shuffle_two_pass(x.data_ptr(), y.data_ptr(), n, 4, SEED, rounds, ws.data_ptr(),
                                             ws.numel(), sp), "bs_probe_shuffle_two_pass")

    def unfused():
        B._check(B.bs_probe_shuffle_unfused(x.data_ptr(), y.data_ptr(), n, 4, SEED, rounds, scratch.data_ptr(),
                                            scratch.numel(), ws.data_ptr(), ws.numel(), sp),
                 "bs_probe_shuffle_unfused")

    def lcg():
        bs.shuffle_lcg(x, SEED, out=y, workspace=ws)

    bs.shuffle(x, SEED, rounds, out=ref, workspace=ws)
    res = {"n": n}
    for name, fn in (("bijective2_fused", fused), ("bijective1_two_pass", two_pass),
                     ("bijective0_unfused", unfused)):
        t = timer.run(fn, 5)
        res[name + "_ms"] = t * 1e3
        res[name + "_Gelem_s"] = n / t / 1e9
        if not torch.equal(y, ref):
            raise RuntimeError(f"fusion form {name} differs from the fused kernel at n={n}")
    t = timer.run(lcg, 5)
    res["lcg_fused_ms"] = t * 1e3
    res["lcg_fused_Gelem_s"] = n / t / 1e9
    # the staged form: the same output through streaming passes
    need = bs.staged_scratch_bytes(n, 4)
    if need:
        st_scratch = torch.empty(need, dtype=torch.uint8, device=dev)
        t = timer.run(lambda: bs.shuffle_staged(x, SEED, rounds, out=y, scratch=st_scratch), 5)
        res["staged_ms"] = t * 1e3
        res["staged_Gelem_s"] = n / t / 1e9
        if not torch.equal(y, ref):
            raise RuntimeError(f"the staged form differs from the fused kernel at n={n}")
        del st_scratch
    # the index-output and inverse variants: the permutation itself (4-byte
    # indices, coalesced writes) and the un-shuffle in its two forms
    # (coalesced reads and scattered writes through f; coalesced writes and
    # gathered reads through f^-1), which must give back x
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    t = timer.run(lambda: bs.permutation(n, SEED, rounds, out=idx, workspace=ws), 5)
    res["permutation_ms"] = t * 1e3
    res["permutation_Gelem_s"] = n / t / 1e9
    bs.shuffle(x, SEED, rounds, out=ref, workspace=ws)
    z = torch.empty_like(x)
    t = timer.run(lambda: bs.unshuffle(ref, SEED, rounds, out=z, workspace=ws), 5)
    res["unshuffle_ms"] = t * 1e3
    res["unshuffle_Gelem_s"] = n / t / 1e9
    if not torch.equal(z, x):
        raise RuntimeError(f"unshuffle did not invert the shuffle at n={n}")
    # the same inverse in gather form through f^-1 (rank table + gather)
    inv_scratch = torch.empty(B.bs_unshuffle_inverse_scratch_bytes(n), dtype=torch.uint8, device=dev)
    z.zero_()
    t = timer.run(lambda: bs.unshuffle_inverse(ref, SEED, rounds, out=z, scratch=inv_scratch), 5)
    res["unshuffle_inverse_ms"] = t * 1e3
    res["unshuffle_inverse_Gelem_s"] = n / t / 1e9
    if not torch.equal(z, x):
        raise RuntimeError(f"unshuffle_inverse did not invert the shuffle at n={n}")
    del inv_scratch
    # and through the staged passes keyed by output position
    need = bs.unshuffle_staged_scratch_bytes(n, 4)
    if need:
        un_scratch = torch.empty(need, dtype=torch.uint8, device=dev)
        z.zero_()
        t = timer.run(lambda: bs.unshuffle_staged(ref, SEED, rounds, out=z, scratch=un_scratch), 5)
        res["unshuffle_staged_ms"] = t * 1e3
        res["unshuffle_staged_Gelem_s"] = n / t / 1e9
        if not torch.equal(z, x):
            raise RuntimeError(f"unshuffle_staged did not invert the shuffle at n={n}")
        del un_scratch
    del idx, z
    perm = torch.randperm(n, device=dev, dtype=torch.int64).to(torch.int32)
    t = timer.run(lambda: B.bs_probe_gather(x.data_ptr(), n, y.data_ptr(), perm.data_ptr(), n, 4, sp), 5)
    res["gather_index_array_ms"] = t * 1e3
    del perm, scratch
    if bs.workspace_error(ws) != 0:
        raise RuntimeError("device-side error in the fusion forms")
    return res


def bench_small(torch, bs, dev, timer) -> dict:
    """The small single-shuffle workload: n = 100,000 uint32 arange, seed 42,
    4 rounds (domain 2^17): launch-bound; per-call time on one stream, eager
    and as 100 calls replayed from one graph."""
    n = 100_000
    x = torch.arange(n, dtype=torch.int32, device=dev)
    y = torch.empty_like(x)
    ws = bs.make_workspace(bs.workspace_bytes(n), device=dev)
    t = timer.run(lambda: bs.shuffle(x, 42, 4, out=y, workspace=ws), 200, warm=10)
    ref = y.clone()
    # the same call 100 times in one captured graph: the device's own time per
    # call, without the host's per-call launch path
    calls = 100
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for _ in range(calls):
            bs.shuffle(x, 42, 4, out=y, workspace=ws)
    torch.cuda.synchronize()
    y.zero_()
    t_graph = timer.run(g.replay, 20, warm=3) / calls
    if not torch.equal(y, ref) or bs.workspace_error(ws) != 0:
        raise RuntimeError("graph replay of the small shuffle differs from the eager call")
    # launch floor for comparison: a 16-byte copy kernel, 100 per graph
    from paper_2106_06161_amd import binding as B

    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=side):
        for _ in range(calls):
            B._check(B.bs_probe_copy(x.data_ptr(), y.data_ptr(), 16, side.cuda_stream), "bs_probe_copy")
    torch.cuda.synchronize()
    t_floor = timer.run(g2.replay, 20, warm=3) / calls
    # dependent device-scope round trips inside a 32-workgroup launch (the
    # small shuffle's tile count): launches of 0, 1, 2, 4 and 8 chained
    # atomics per workgroup, 100 per graph
    words = torch.zeros(128, dtype=torch.int32, device=dev)
    trips = {}
    for chain in (0, 1, 2, 4, 8):
        g3 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g3, stream=side):
            for _ in range(calls):
                B._check(B.bs_probe_round_trips(words.data_ptr(), 32, chain, side.cuda_stream),
                         "bs_probe_round_trips")
        torch.cuda.synchronize()
        trips[chain] = timer.run(g3.replay, 20, warm=3) / calls * 1e6
        del g3
    del g, g2
    return {"workload": "n=100,000 uint32 arange, seed 42, 4 rounds, domain 2^17", "us_per_call": t * 1e6,
            "Gelem_s": n / t / 1e9, "us_per_call_graph": t_graph * 1e6, "Gelem_s_graph": n / t_graph / 1e9,
            "graph_launch_floor_us": t_floor * 1e6,
            "round_trip_launch_us_by_chain": trips,
            "round_trip_us": (trips[8] - trips[0]) / 8}


FOOTPRINTS_MIB = [32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]


def random_read_rate(B, torch, timer, buf, region_bytes: int, eb: int, reads: int, sp) -> float:
    """Random reads per second (G/s) of eb-byte records at hashed indices over
    region_bytes of buf (bs_probe_random_reads_region)."""
    out = torch.empty(reads // 16, dtype=torch.int32, device=buf.device)
    t = timer.run(lambda: B._check(B.bs_probe_random_reads_region(buf.data_ptr(), region_bytes, eb, reads,
                                                                  out.data_ptr(), 3, sp),
                                   "bs_probe_random_reads_region"), 5)
    del out
    return reads / t / 1e9


def bench_footprint(torch, B, dev, stream, timer) -> list:
    """The random-read ceiling against the region read (32 MiB .. 8 GiB) and
    the record size (4, 8, 16 B): 2^27 reads per point."""
    sp = stream.cuda_stream
    buf = torch.zeros(FOOTPRINTS_MIB[-1] << 18, dtype=torch.int32, device=dev)
    rows = []
    for eb in (4, 8, 16):
        for mib in FOOTPRINTS_MIB:
            log(f"bench: random reads, {eb}-byte records over {mib} MiB")
            rate = random_read_rate(B, torch, timer, buf, mib << 20, eb, 1 << 27, sp)
            rows.append({"elem_bytes": eb, "region_MiB": mib, "G_reads_s": rate, "GBps_useful": rate * eb})
    del buf
    return rows


def bench_large(torch, bs, B, dev, stream, timer, rounds) -> dict:
    """n = 10^9 uint32 arange (seed 1, domain 2^30) and 2.5e8 records of four
    float32 (seeded device normal values, seed 11, domain 2^28): bs_shuffle as
    a caller gets it (a workspace with room for the staged form; the tuned
    table picks the form), and each form explicitly, beside the random-read
    ceiling over the same footprint (4 GiB) and record size."""
    sp = stream.cuda_stream
    res = {}
    probe = torch.zeros(1 << 30, dtype=torch.int32, device=dev)  # 4 GiB
    for name, eb in (("u32", 4), ("rec16", 16)):
        res[f"ceiling_{name}_4GiB_G_reads_s"] = random_read_rate(B, torch, timer, probe, 4 << 30, eb, 1 << 28, sp)
    del probe
    for name, n, make, seed in (("u32_1e9", 10**9, lambda n: torch.arange(n, dtype=torch.int32, device=dev), 1),
                                ("rec16_2p5e8", 250_000_000,
                                 lambda n: torch.randn((n, 4), dtype=torch.float32, device=dev,
                                                       generator=torch.Generator(device=dev).manual_seed(11)), 11)):
        log(f"bench: large {name}")
        x = make(n)
        y = torch.empty_like(x)
        eb = x.element_size() * (x.numel() // n)
        ws = bs.make_workspace(bs.workspace_bytes(n, elem_bytes=eb, staged=True), device=dev)
        t = timer.run(lambda: bs.shuffle(x, seed, rounds, out=y, workspace=ws), 3)
        ref = y.clone()
        launch = list(B.bs_query_config(0, eb, n))
        res[f"{name}_form"] = "staged" if launch[2] == DEPTH_STAGED else "fused"
        res[f"{name}_launch"] = launch
        res[f"{name}_ms"] = t * 1e3
        res[f"{name}_Gelem_s"] = n / t / 1e9
        res[f"{name}_alg_GBps"] = 2.0 * eb * n / t / 1e9
        fws = bs.make_workspace(bs.workspace_bytes(n), device=dev)
        tf = timer.run(lambda: bs.shuffle(x, seed, rounds, out=y, workspace=fws), 3)
        if not torch.equal(y, ref):
            raise RuntimeError(f"the fused kernel differs from bs_shuffle's form at {name}")
        res[f"{name}_fused_ms"] = tf * 1e3
        ceil = res["ceiling_u32_4GiB_G_reads_s" if eb == 4 else "ceiling_rec16_4GiB_G_reads_s"]
        res[f"{name}_fused_pct_of_same_footprint_ceiling"] = 100.0 * (n / tf / 1e9) / ceil
        need = bs.staged_scratch_bytes(n, eb)
        if need:
            scratch = torch.empty(need, dtype=torch.uint8, device=dev)
            ts = timer.run(lambda: bs.shuffle_staged(x, seed, rounds, out=y, scratch=scratch), 3)
            if not torch.equal(y, ref):
                raise RuntimeError(f"the staged form differs from bs_shuffle's form at {name}")
            res[f"{name}_staged_ms"] = ts * 1e3
            res[f"{name}_staged_Gelem_s"] = n / ts / 1e9
            del scratch
        if bs.workspace_error(ws) != 0 or bs.workspace_error(fws) != 0:
            raise RuntimeError(f"device-side error in the large workload {name}")
        del x, y, ref, ws, fws
        torch.cuda.empty_cache()
    return res


def bench_sweep(torch, bs, B, dev, stream, timer, rounds, gather: bool = False) -> list:
    """Sec. 6's protocol on this chip: the fused kernel over n = 2^w and
    2^w + 1, w = 8..30, for 4- and 8-byte records (mean of 5 launches), beside
    the random-read ceiling at the same record size over a region of 2^w
    records (the same footprint), and optionally a random gather with an
    index array."""
    out = []
    sp = stream.cuda_stream
    for eb, dt in ((4, torch.int32), (8, torch.int64)):
        for w in range(8, 31):
            x = torch.arange((1 << w) + 1, dtype=torch.int64, device=dev).to(dt)
            y = torch.empty_like(x)
            ws = bs.make_workspace(bs.workspace_bytes((1 << w) + 1, elem_bytes=eb, staged=True), device=dev)
            reads = max(1 << 16, ((1 << w) + 15) // 16 * 16)
            ceil = random_read_rate(B, torch, timer, x, (1 << w) * eb, eb, reads, sp)
            for n in (1 << w, (1 << w) + 1):
                log(f"bench: sweep elem_bytes={eb} n={n}")
                xs, ys = x[:n], y[:n]
                t = timer.run(lambda: bs.shuffle(xs, SEED, rounds, out=ys, workspace=ws), 5)
                launch = list(B.bs_query_config(0, eb, n))
                row = {"elem_bytes": eb, "n": n, "shuffle_ms": t * 1e3, "Gelem_s": n / t / 1e9,
                       "random_read_ceiling_G_s": ceil, "pct_of_ceiling": 100.0 * (n / t / 1e9) / ceil,
                       "form": "staged" if launch[2] == DEPTH_STAGED else "fused", "launch": launch}
                if gather:
                    idx = torch.randperm(n, device=dev, dtype=torch.int64).to(torch.int32)
                    tg = timer.run(lambda: B.bs_probe_gather(xs.data_ptr(), n, ys.data_ptr(), idx.data_ptr(), n,
                                                             eb, sp), 5)
                    row["gather_ms"] = tg * 1e3
                    del idx
                out.append(row)
            if bs.workspace_error(ws) != 0:
                raise RuntimeError("device-side error in the sweep")
            del x, y, ws
            torch.cuda.empty_cache()
    return out


def bench_serving(rounds: int, count: int, loads) -> dict:
    """The continuous-batching server on `count` requests: closed-loop
    capacity C (every request arrives at once), then Poisson arrivals at each
    fraction of C in `loads`.  Admission budget: the device's free memory."""
    from paper_2106_06161_amd.serve import HipExecutor, ShuffleServer, make_requests

    ex = HipExecutor(streams=4, rounds=rounds, pool_items=1 << 27)
    srv = ShuffleServer(ex)
    cap = srv.run(make_requests(count, 1000, 100_000_000, qps=1e12, seed=5)).summary()
    log(f"bench: serving closed loop {cap['requests_per_s']:.0f} requests/s, {cap['failed']} failed")
    res = {
        "workload": f"{count} requests per run, sizes floor(exp(U(ln 1e3, ln 1e8))), dtype uniform over "
                    "uint32/int64/float32, 64-bit seeds (PCG64 5, then 6); payloads resident in HBM; admission "
                    "budget = free device memory at the start of each run; 4 streams, requests <= 2^20 records "
                    "coalesced",
        "closed_loop": cap,
        "open_loop": [],
    }
    for f in loads:
        qps = f * cap["requests_per_s"]
        run = srv.run(make_requests(count, 1000, 100_000_000, qps=qps, seed=6)).summary()
        log(f"bench: serving at {f} C: p50 {run['latency_p50_ms']:.2f} ms, p99 {run['latency_p99_ms']:.2f} ms, "
            f"{run['failed']} failed")
        res["open_loop"].append(dict(run, load=f, qps=qps))
    res["p50_ms"] = {str(r["load"]): r["latency_p50_ms"] for r in res["open_loop"]}
    res["p99_ms"] = {str(r["load"]): r["latency_p99_ms"] for r in res["open_loop"]}
    res["device_error"] = int(ex.check_errors())
    return res


def main() -> int:
    args = parse_args()
    if args.traffic_record:
        print(json.dumps(traffic_record(args.traffic_record), indent=1))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the shuffle runs on a single device)", flush=True)
        return 2
    import numpy as np
    import torch

    import paper_2106_06161_amd as bs
    from paper_2106_06161_amd import binding as B
    from paper_2106_06161_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    timer = Timer(torch, stream)
    rounds = args.rounds

    if args.profile_small:
        small = bench_small(torch, bs, dev, timer)
        log(f"bench: small workload {json.dumps(small)}")
        print(json.dumps({"small": small}), flush=True)
        return 0
    if args.profile_batched:
        b = W.batch(4096, 100, 1_000_000, seed=3)
        total = b["total"]
        xb = torch.arange(total, dtype=torch.int64, device=dev).to(torch.int32)
        yb = torch.empty_like(xb)
        off = torch.from_numpy(b["offsets"]).to(dev)
        sd = torch.from_numpy(b["seeds"].view(np.int64)).to(dev)
        wsb = bs.make_workspace(bs.workspace_bytes(total, 4096), device=dev)
        for _ in range(args.warmup + args.steps):
            bs.shuffle_batched(xb, off, sd, rounds, out=yb, workspace=wsb)
        torch.cuda.synchronize()
        err = bs.workspace_error(wsb)
        log(f"bench: {args.warmup + args.steps} batched launches, launch {B.bs_query_config(1, 4, total, 4096)}, "
            f"device status {err}")
        return 1 if err else 0

    if args.profile_footprint:
        nb = 512 << 20
        src = torch.zeros(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        B._check(B.bs_probe_copy(src.data_ptr(), dst.data_ptr(), nb, sp), "bs_probe_copy")
        torch.cuda.synchronize()
        del src, dst
        rows = bench_footprint(torch, B, dev, stream, timer)
        print(json.dumps({"footprint": rows}), flush=True)
        return 0

    if args.profile_large:
        nb = 512 << 20
        src = torch.zeros(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        B._check(B.bs_probe_copy(src.data_ptr(), dst.data_ptr(), nb, sp), "bs_probe_copy")
        torch.cuda.synchronize()
        del src, dst
        res = {}
        for name, n, shape, dt, seed in (("u32_1e9", 10**9, (10**9,), torch.int32, 1),
                                         ("rec16_2p5e8", 250_000_000, (250_000_000, 4), torch.float32, 11),
                                         ("u64_2p27p1", N_HEADLINE, (N_HEADLINE,), torch.int64, SEED)):
            log(f"bench: profile {name}")
            x = torch.zeros(shape, dtype=dt, device=dev)
            y = torch.empty_like(x)
            ws = bs.make_workspace(bs.workspace_bytes(n), device=dev)
            for _ in range(args.steps):
                bs.shuffle(x, seed, rounds, out=y, workspace=ws)
            torch.cuda.synchronize()
            if bs.workspace_error(ws) != 0:
                raise RuntimeError(f"device-side error in {name}")
            res[name] = list(B.bs_query_config(0, x.element_size() * (x.numel() // n), n))
            del x, y, ws
        print(json.dumps({"launch": res}), flush=True)
        return 0

    if args.profile_unshuffle:
        x = torch.from_numpy(W.uniform_u32(N_HEADLINE, seed=SEED)).to(dev)
        shuffled = bs.shuffle(x, SEED, rounds)
        back = torch.empty_like(x)
        scratch = torch.empty(bs.unshuffle_staged_scratch_bytes(N_HEADLINE, 4), dtype=torch.uint8, device=dev)
        for _ in range(args.warmup + args.steps):
            bs.unshuffle_staged(shuffled, SEED, rounds, out=back, scratch=scratch)
        torch.cuda.synchronize()
        if not torch.equal(back, x):
            log("bench: the staged un-shuffle did not give the input back")
            return 1
        log(f"bench: {args.warmup + args.steps} staged un-shuffles of n={N_HEADLINE}")
        return 0
    if args.profile_staged:
        n = 10**9 if args.staged_large else N_HEADLINE
        x = torch.from_numpy(W.uniform_u32(n, seed=SEED)).to(dev)
        y = torch.empty_like(x)
        B._check(B.bs_probe_copy(x.data_ptr(), y.data_ptr(), (N_HEADLINE * 4) // 16 * 16, sp), "bs_probe_copy")
        scratch = torch.empty(bs.staged_scratch_bytes(n, 4), dtype=torch.uint8, device=dev)
        for _ in range(args.warmup + args.steps):
            bs.shuffle_staged(x, SEED, rounds, out=y, scratch=scratch)
        torch.cuda.synchronize()
        log(f"bench: {args.warmup + args.steps} staged shuffles of n={n}")
        return 0

    log("bench: generating the headline input (n=2^27+1 uint32, PCG64 seed 7)")
    x_np = W.uniform_u32(N_HEADLINE, seed=SEED)
    x = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(x)
    # the product call: bs_shuffle with room for either form (it takes the
    # staged form where the tuned table prefers it)
    ws = bs.make_workspace(bs.workspace_bytes(N_HEADLINE, staged=True), device=dev)

    if args.profile:
        nb = (N_HEADLINE * 4) // 16 * 16
        B._check(B.bs_probe_copy(x.data_ptr(), y.data_ptr(), nb, sp), "bs_probe_copy")
        torch.cuda.synchronize()
        log(f"bench: copy probe of {nb} bytes done")

    def step():
        bs.shuffle(x, SEED, rounds, out=y, workspace=ws)

    log(f"bench: {args.warmup} warmup steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: exactly K steps, synchronized on both sides
    log(f"bench: timing {args.steps} steps")
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev0[i].record(stream)
        step()
        ev1[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = sorted(a.elapsed_time(b) for a, b in zip(ev0, ev1))
    kernel_s = sum(per_step) / args.steps * 1e-3
    err = bs.workspace_error(ws)
    if err != 0:
        log(f"bench: device-side error {B.status_string(err)}")
        return 1
    log(f"bench: {wall / args.steps * 1e3:.3f} ms/step wall, {kernel_s * 1e3:.3f} ms kernel")
    y_timed = y.cpu().numpy()  # the timed steps' output, checked whole against the oracle in the CPU leg

    alg_bytes = 2 * 4 * N_HEADLINE
    achieved = alg_bytes / kernel_s / 1e9
    digest = kernel_source_digest()
    launch = dict(zip(("waves", "items", "depth", "grid_mult"), B.bs_query_config(0, 4, N_HEADLINE)))
    form = "staged" if launch["depth"] == DEPTH_STAGED else "fused"
    traffic = committed_traffic(digest, launch, rounds)
    result = {
        "metric": "Gelem/s + % HBM peak at n=2^27+1 u32; batched vs per-call; p99 latency",
        "value": N_HEADLINE * args.steps / wall / 1e9,
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "single bijective shuffle, n=2^27+1 uint32 uniform (PCG64 seed 7), seed 7, "
                        f"{rounds} rounds, domain 2^28",
            "n": N_HEADLINE, "elem_bytes": 4, "rounds": rounds, "seed": SEED,
            "launch": launch, "form": form,
        },
        "pct_hbm_peak": 100.0 * (alg_bytes * args.steps / wall / 1e9) / HBM_PEAK_GBPS,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic["hbm_bytes_per_launch"] if traffic else None,
            "kernel": kernel_label(launch, rounds),
            "kernel_ms": kernel_s * 1e3,
            "kernel_ms_median": per_step[len(per_step) // 2],
            "kernel_ms_min": per_step[0],
            "algorithmic_bytes_per_launch": alg_bytes,
            "kernel_source_digest": digest,
        },
    }
    if traffic:
        # FETCH_SIZE and WRITE_SIZE count what the L2s exchange with the data
        # fabric; the fabric serves part of it from the Infinity Cache, so
        # this is an upper bound on DRAM traffic, not DRAM traffic
        result["roofline"]["l2_fabric_GBps"] = traffic["hbm_bytes_per_launch"] / kernel_s / 1e9
        result["roofline"]["fetch_bytes_per_elem"] = traffic["fetch_bytes_per_launch"] / N_HEADLINE
        result["roofline"]["write_bytes_per_elem"] = traffic["write_bytes_per_launch"] / N_HEADLINE
        result["roofline"]["traffic_kernel_ms_rocprof"] = traffic["kernel_avg_ms_rocprof"]
    if args.profile:
        print(json.dumps(result), flush=True)
        return 0

    if not args.no_ceilings:
        log("bench: ceilings (copy, random gather, cipher+scan alone, variants)")
        ceil = {}
        nb = (N_HEADLINE * 4) // 16 * 16
        t = timer.run(lambda: B.bs_probe_copy(x.data_ptr(), y.data_ptr(), nb, sp), 10)
        ceil["copy_GBps"] = 2 * nb / t / 1e9
        perm = torch.randperm(N_HEADLINE, device=dev, dtype=torch.int64).to(torch.int32)
        t = timer.run(lambda: B.bs_probe_gather(x.data_ptr(), N_HEADLINE, y.data_ptr(), perm.data_ptr(),
                                                N_HEADLINE, 4, sp), 10)
        del perm
        ceil["gather_index_array_ms"] = t * 1e3
        ceil["gather_index_array_Gelem_s"] = N_HEADLINE / t / 1e9
        # random 4-byte reads over 512 MiB at hashed indices, 16 in flight per lane
        words = 1 << 27
        sums = torch.empty(words // 16, dtype=torch.int32, device=dev)
        t = timer.run(lambda: B._check(B.bs_probe_random_reads(x.data_ptr(), words, sums.data_ptr(), 3, sp),
                                       "bs_probe_random_reads"), 10)
        del sums
        ceil["random_reads_512MiB_ms"] = t * 1e3
        ceil["random_reads_512MiB_G_s"] = words / t / 1e9
        t = timer.run(lambda: B.bs_probe_cipher_scan(N_HEADLINE, SEED, rounds, ws.data_ptr(), ws.numel(), sp), 10)
        ceil["cipher_scan_only_ms"] = t * 1e3
        t = timer.run(lambda: B.bs_probe_cipher_scan(N_HEADLINE, SEED, 4, ws.data_ptr(), ws.numel(), sp), 10)
        ceil["cipher_scan_only_4_rounds_ms"] = t * 1e3
        t4 = timer.run(lambda: bs.shuffle(x, SEED, 4, out=y, workspace=ws), 10)
        ceil["shuffle_4_rounds_ms"] = t4 * 1e3
        ceil["shuffle_4_rounds_Gelem_s"] = N_HEADLINE / t4 / 1e9
        xp, yp = x[: 1 << 27], y[: 1 << 27]
        tp = timer.run(lambda: bs.shuffle(xp, SEED, rounds, out=yp, workspace=ws), 10)
        ceil["shuffle_pow2_n2p27_ms"] = tp * 1e3
        ceil["shuffle_pow2_n2p27_Gelem_s"] = (1 << 27) / tp / 1e9
        # integer VALU issue rates (the cipher's instructions): SIMD cycles per
        # wave instruction at 2.4 GHz over 1,024 SIMDs; 4 is one wave64
        # instruction per 4 cycles on a 16-lane SIMD (full rate)
        groups, iters = 2048, 4096
        sink = torch.empty(groups * 256, dtype=torch.int32, device=dev)
        rates = {}
        for op, name in enumerate(("v_xor_b32", "v_mul_u32_u24", "v_mad_u32_u24", "v_mul_lo_u32", "v_mul_hi_u32",
                                   "v_mad_u64_u32+v_xor_b32")):
            t = timer.run(lambda: B._check(B.bs_probe_int_rate(op, iters, sink.data_ptr(), groups, sp),
                                           "bs_probe_int_rate"), 5)
            rates[name] = t * 2.4e9 * 1024 / (groups * 4 * iters * 8)
        del sink
        ceil["int_valu_cycles_per_wave_instruction"] = rates
        ceil["shuffle_pct_of_copy"] = 100.0 * achieved / ceil["copy_GBps"]
        ceil["shuffle_pct_of_gather"] = 100.0 * ceil["gather_index_array_ms"] / (kernel_s * 1e3)
        ceil["shuffle_pct_of_random_read_rate"] = 100.0 * (N_HEADLINE / kernel_s / 1e9) / ceil["random_reads_512MiB_G_s"]
        result["ceilings"] = ceil
        if bs.workspace_error(ws) != 0:
            log("bench: device-side error in ceilings")
            return 1

    if not args.no_fusion:
        log("bench: fusion forms at the headline size (fused, two-pass scan, unfused, LCG)")
        result["fusion"] = bench_fusion(torch, bs, B, W, dev, stream, timer, rounds, N_HEADLINE, x, y)
        if args.fusion_sweep:
            sweep = []
            for bits in range(20, 30):
                for n in (1 << bits, (1 << bits) + 1):
                    log(f"bench: fusion sweep n={n}")
                    sweep.append(bench_fusion(torch, bs, B, W, dev, stream, timer, rounds, n))
            result["fusion_sweep"] = sweep

    if not args.no_large:
        log("bench: small (n=100,000, 4 rounds) and large (10^9 uint32; 2.5e8 x 16-byte records) workloads")
        result["small"] = bench_small(torch, bs, dev, timer)
        result["large"] = bench_large(torch, bs, B, dev, stream, timer, rounds)
    if not args.no_ceilings:
        log("bench: random-read ceiling against footprint and record size")
        result["random_reads_by_footprint"] = bench_footprint(torch, B, dev, stream, timer)
    if not args.no_sweep:
        log("bench: size sweep (n = 2^w and 2^w+1, w = 8..30; uint32 and uint64)")
        result["sweep"] = bench_sweep(torch, bs, B, dev, stream, timer, rounds, gather=args.gather_sweep)

    if not args.no_batched:
        log("bench: batched vs per-call (4,096 segments, log-uniform sizes in [100, 10^6], PCG64 seed 3)")
        result["batched"] = bench_batched(torch, bs, W, np, dev, stream, timer, rounds)
        log("bench: batches of small segments (100,000 permutations of n = 5 / 100 / 1,000; 65,536 segments)")
        result["batched_small"] = bench_batched_small(torch, bs, B, W, np, dev, timer, rounds)

    if not args.no_serving:
        log(f"bench: serving ({args.serve_requests} requests, sizes log-uniform in [10^3, 10^8], "
            "dtype uniform over uint32/int64/float32)")
        loads = [float(v) for v in args.serve_loads.split(",") if v]
        result["serving"] = bench_serving(rounds, args.serve_requests, loads)

    if not args.no_cpu_baseline:
        log("bench: CPU baseline (oracle, one thread, bounded sample) and std::shuffle")
        result["cpu_baseline"] = cpu_baseline(x_np, y_timed)
        result["cpu_std_shuffle"] = cpu_std_shuffle(x_np)
        if not result["cpu_baseline"]["gpu_output_equal"]:
            log("bench: the timed GPU output differs from the oracle's")
            print(json.dumps(result), flush=True)
            return 1
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
