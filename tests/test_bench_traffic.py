"""The measurement pipeline's host arithmetic: bench.py --traffic-record turns
rocprofv3 CSVs into the traffic record that the roofline reads (FETCH_SIZE and
WRITE_SIZE scaled by a copy of known size), and bench.py only uses a record
whose kernel sources and launch shape match.  Synthetic CSVs, CPU only."""
import csv
import json
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

KERNEL = "void bsd::shuffle_compact_kernel<4, false, 16, 16, true, 0, true, false>(bsd::SingleArgs)"
COPY = "void (anonymous namespace)::copy16_kernel(unsigned int const*, unsigned int*, unsigned long)"
LAUNCH = {"waves": 16, "items": 16, "depth": 9, "grid_mult": 1}


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, name, copy_value, kernel_values):
    rows = [[COPY, name, copy_value]] + [[KERNEL, name, v] for v in kernel_values]
    _write(os.path.join(d, "x_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)


@pytest.fixture
def runs(tmp_path):
    kt = str(tmp_path / "kt")
    _write(os.path.join(kt, "kt_kernel_stats.csv"), ["Name", "Calls", "AverageNs"],
           [[KERNEL, 12, 2_440_000.0], [COPY, 1, 200_000.0]])
    copy_bytes = ((bench.N_HEADLINE * 4) // 16) * 16
    # the copy's counter reads half its bytes for FETCH (scale 2) and all for WRITE (scale 1)
    _counters(str(tmp_path / "fetch"), "FETCH_SIZE", copy_bytes / 2 / 1024, [1000.0, 3000.0])
    _counters(str(tmp_path / "write"), "WRITE_SIZE", copy_bytes / 1024, [500.0])
    _counters(str(tmp_path / "sq"), "SQ_INSTS_VALU", 1.0, [10.0, 30.0])
    _counters(str(tmp_path / "tcc"), "TCC_EA0_RDREQ_sum", 7.0, [5.0])
    js = tmp_path / "kt.json"
    js.write_text("log line\n" + json.dumps({"config": {"launch": LAUNCH}}) + "\n")
    return [kt, str(tmp_path / "fetch"), str(tmp_path / "write"), str(js), str(tmp_path / "sq"),
            str(tmp_path / "tcc")]


def test_traffic_record_scales_counters_by_the_copy(runs):
    rec = bench.traffic_record(runs)
    assert rec["fetch_scale_from_copy"] == pytest.approx(2.0)
    assert rec["write_scale_from_copy"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)  # mean of 1000 and 3000 KiB
    assert rec["write_bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])
    assert rec["kernel_avg_ms_rocprof"] == pytest.approx(2.44)
    assert rec["kernel_calls_rocprof"] == 12
    assert rec["launch"] == LAUNCH
    assert rec["sq_insts_valu_per_launch"] == pytest.approx(20.0)
    assert rec["tcc_ea0_rdreq_sum_per_launch"] == pytest.approx(5.0)
    assert rec["tcc_ea0_rdreq_sum_copy"] == pytest.approx(7.0)
    assert rec["kernel_source_digest"] == bench.kernel_source_digest()


def test_record_is_used_only_for_matching_sources_and_shape(runs, tmp_path, monkeypatch):
    rec = bench.traffic_record(runs)
    path = tmp_path / "traffic.txt"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    digest = bench.kernel_source_digest()
    assert bench.committed_traffic(digest, LAUNCH)["hbm_bytes_per_launch"] == rec["hbm_bytes_per_launch"]
    assert bench.committed_traffic("0" * 16, LAUNCH) is None
    assert bench.committed_traffic(digest, dict(LAUNCH, grid_mult=0)) is None
    assert bench.committed_traffic(digest, LAUNCH, rounds=4) is None  # the record is of 24 rounds


def test_traffic_record_sums_the_staged_passes(tmp_path):
    """A staged step runs several kernels once each: the record sums their
    per-launch averages (time, FETCH, WRITE)."""
    names = ["void bsd::(anonymous namespace)::staged_first_kernel<4, false>(bsd::StagedArgs)",
             "void bsd::(anonymous namespace)::staged_second_kernel<4>(bsd::StagedArgs)",
             "void bsd::(anonymous namespace)::staged_place_kernel<4>(bsd::StagedArgs)"]
    kt = str(tmp_path / "kt")
    _write(os.path.join(kt, "kt_kernel_stats.csv"), ["Name", "Calls", "AverageNs"],
           [[names[0], 5, 800_000.0], [names[1], 5, 500_000.0], [names[2], 5, 400_000.0], [COPY, 1, 1.0]])
    copy_bytes = ((bench.N_HEADLINE * 4) // 16) * 16
    for d, name, scale in (("fetch", "FETCH_SIZE", 2), ("write", "WRITE_SIZE", 1)):
        rows = [[COPY, name, copy_bytes / scale / 1024]]
        rows += [[nm, name, 100.0 * (i + 1)] for i, nm in enumerate(names) for _ in range(2)]
        _write(os.path.join(str(tmp_path / d), "x_counter_collection.csv"),
               ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    js = tmp_path / "kt.json"
    launch = {"waves": 0, "items": 0, "depth": 16, "grid_mult": 0}
    js.write_text(json.dumps({"config": {"launch": launch}}) + "\n")
    rec = bench.traffic_record([kt, str(tmp_path / "fetch"), str(tmp_path / "write"), str(js)])
    assert rec["kernel_avg_ms_rocprof"] == pytest.approx(1.7)
    assert rec["fetch_bytes_per_launch"] == pytest.approx((100 + 200 + 300) * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx((100 + 200 + 300) * 1024 * 1.0)
    assert len(rec["per_kernel_ms_rocprof"]) == 3 and rec["launch"] == launch


def test_kernel_label_follows_the_first_pass_shape():
    staged = {"waves": 0, "items": 0, "depth": bench.DEPTH_STAGED, "grid_mult": 0}
    assert "staged_first_kernel<4, false, true>" in bench.kernel_label(staged, 24)
    assert "staged_first_kernel<4, false, false>" in bench.kernel_label(staged, 4)
    assert bench.kernel_label(staged).count(" + ") == 4
