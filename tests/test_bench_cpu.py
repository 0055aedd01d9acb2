"""The measurement reduction behind profiles/ (bench.py --summarize) on
synthetic rocprofv3 CSV files of known content: the copy calibration, the
working-launch medians, the traffic sum and the VALU issue bound, and the two
readers the bench line takes its traffic and rocprofv3 average from."""
import csv
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

KERNEL = "void topo::k_cg_matvec1<float, false, false, 1>"
SUMMARY = "kernel_trace_cg_256x128x128.txt"


def _write(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def _counters(path, kernel, counter, values):
    _write(path, ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [{"Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": v} for v in values])


@pytest.fixture
def runs(tmp_path):
    root = tmp_path / "prof" / "host" / "1234"
    root.mkdir(parents=True)
    copy = "__amd_rocclr_copyBuffer"
    kib = bench.COPY_BYTES / 1024.0
    # the copy reads COPY_BYTES: FETCH_SIZE reads half of it (scale 2), WRITE_SIZE all (scale 1)
    _counters(root / "copy_fetch_counter_collection.csv", copy, "FETCH_SIZE", [kib / 2] * 3)
    _counters(root / "copy_write_counter_collection.csv", copy, "WRITE_SIZE", [kib] * 3)
    full = KERNEL + "(double*, int*, double const*)"
    # four launches after the solve stopped (no work), four working ones
    durs = [1.0, 1.0, 1.0, 1.0, 50.0, 60.0, 70.0, 80.0]
    t, rows = 10 ** 9, []
    for d in durs:
        rows.append({"Kernel_Name": full, "Start_Timestamp": t, "End_Timestamp": t + int(d * 1e3)})
        t += 10 ** 6
    _write(root / "cg3_trace_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           rows)
    _counters(root / "cg3_fetch_counter_collection.csv", full, "FETCH_SIZE", [10, 10, 1000, 1000])
    _counters(root / "cg3_write_counter_collection.csv", full, "WRITE_SIZE", [5, 5, 500, 500])
    # 30 us of VALU issue: 30 us x 2400 cycles/us x 256 CUs
    _counters(root / "cg3_sq_counter_collection.csv", full, "SQ_INSTS_VALU", [256 * 2400 * 30] * 2)
    out = tmp_path / "profiles"
    out.mkdir()
    return tmp_path / "prof", out


def _fields(text, kernel):
    for sec in text.split("## ")[1:]:
        f = dict(l.split(": ", 1) for l in sec.splitlines() if ": " in l)
        if f.get("kernel") == kernel:
            return f
    raise AssertionError("no section for " + kernel)


def test_summarize_reduces_counters_and_durations(runs):
    root, out = runs
    bench.summarize(str(root), str(out))
    cal = (out / "pmc_copy_calibration.txt").read_text()
    assert "fetch_scale: 2.0000" in cal and "write_scale: 1.0000" in cal
    assert sorted(os.listdir(out)) == ["kernel_trace_cg_256x128x128.txt", "pmc_copy_calibration.txt"]
    text = (out / SUMMARY).read_text()
    f = _fields(text, KERNEL)
    # avg over all 8 launches; working median = median of the upper half (50..80)
    assert f["launches"].startswith("8, avg_us: 33.000, working_median_us: 65.000")
    # per dispatch: FETCH 1000 KiB x 2 + WRITE 500 KiB x 1
    assert f["traffic_bytes_per_launch"] == str(1024 * (1000 * 2 + 500))
    alg = bench.algorithmic_bytes(KERNEL.split("::")[1], bench.LARGE)
    assert f["algorithmic_bytes_per_launch"] == str(alg)
    assert f["traffic_over_algorithmic"] == "%.3f" % (1024 * 2500 / alg)
    assert f["valu_issue_us_lower_bound"] == "30.0 (0.46 of the working median)"
    assert bench._source_sha(bench.PRODUCT_SOURCES) in f["source"]


def test_bench_readers_take_the_summary_and_reject_stale_sources(runs, monkeypatch):
    root, out = runs
    bench.summarize(str(root), str(out))
    assert bench.measured_traffic(SUMMARY, KERNEL, str(out)) == 1024 * 2500
    assert bench.profiled_avg_us(SUMMARY, KERNEL, str(out)) == pytest.approx(33.0)
    assert bench.profiled_avg_us(SUMMARY, KERNEL.replace("1>", "0>"), str(out)) is None
    # counters taken on other kernel sources are not used
    monkeypatch.setattr(bench, "_source_sha", lambda files: "0123456789abcdef")
    assert bench.measured_traffic(SUMMARY, KERNEL, str(out)) is None
    assert bench.profiled_avg_us(SUMMARY, KERNEL, str(out)) is None

