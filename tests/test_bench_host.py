"""Host-side logic of bench.py (no GPU): the single-GPU contract, the counter
summaries the roofline's traffic comes from, and the source-hash guard that
drops counters taken from other kernel sources."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr and p.stdout == ""


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path):
    kern = "void hs::(anonymous namespace)::k_sum_xcd<32, true, false, 2>(hs::XcdArgs)"
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>"
    calib_kib = bench.CALIB_BYTES / 1024.0
    # the copy reads half of what it moves (factor 2), the kernel 1000 KiB per dispatch
    _counter_csv(str(tmp_path / "fetch"), [(neg, "FETCH_SIZE", calib_kib / 2), (kern, "FETCH_SIZE", 1000.0),
                                           (kern, "FETCH_SIZE", 1000.0)])
    _counter_csv(str(tmp_path / "write"), [(neg, "WRITE_SIZE", calib_kib), (kern, "WRITE_SIZE", 10.0)])
    out = bench.pmc_summary([str(tmp_path / "fetch"), str(tmp_path / "write")])
    recs = [json.loads(l[6:]) for l in out.splitlines() if l.startswith("json: ")]
    assert len(recs) == 1
    r = recs[0]
    assert r["kernel"] == "k_sum_xcd<32, true, false, 2>" and r["source"] == bench.source_hash()
    assert r["fetch_bytes"] == pytest.approx(2 * 1000.0 * 1024)
    assert r["write_bytes"] == pytest.approx(10.0 * 1024)


def test_profile_records_follow_the_sources(tmp_path):
    good = {"kernel": "k_presto<32, 2, false>", "file": "hs_presto.hip",
            "source": bench.source_hash("hs_presto.hip"), "valu": 1.0, "fetch_bytes": 2.0, "write_bytes": 3.0}
    greedy = dict(good, kernel="k_sum_1d<16, true, false>", file="hs_sum.hip", source=bench.source_hash("hs_sum.hip"))
    stale = dict(good, kernel="k_presto<32, 3, false>", source="0000000000000000")
    f = tmp_path / "t2.txt"
    f.write_text("# summary\njson: %s\njson: %s\njson: %s\n" % (json.dumps(good), json.dumps(stale), json.dumps(greedy)))
    recs = bench.profile_records(str(f))
    assert sorted(k for _, k in recs) == ["k_presto<32, 2, false>", "k_sum_1d<16, true, false>"]
    assert bench.read_counters("k_presto<32, 3, false>", str(f)) is None


def test_work_and_line_counts_follow_the_truncation_rule():
    # greedy: fundamental n sums min(H, (N-1)//(n+1)) harmonics; fundamental_end bounds n
    N, H = 1000, 8
    want = sum(min(H, (N - 1) // (n + 1)) for n in range(1, N))
    assert bench.keff_sum([N], H, True) == want
    want_end = sum(min(H, (N - 1) // (n + 1)) for n in range(1, 100))
    assert bench.keff_sum([N], H, True, fundamental_end=100) == want_end
    lines = sum(min(4 * k, 128) for n in range(1, N) for k in range(1, min(H, (N - 1) // (n + 1)) + 1))
    assert bench.line_bytes_sum([N], H, True, 4) == lines


def test_kernel_trace_durations_are_summarised(tmp_path):
    d = tmp_path / "trace"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs"])
        w.writerow(["void hs::(anonymous namespace)::k_sum_xcd<32, true, false, 4>(hs::XcdArgs)", 4, 40000000, 10000000])
    out = bench.pmc_summary([str(d)])
    recs = [json.loads(l[6:]) for l in out.splitlines() if l.startswith("json: ")]
    assert len(recs) == 1 and recs[0]["kernel"] == "k_sum_xcd<32, true, false, 4>"
    assert recs[0]["avg_ns"] == pytest.approx(1e7) and recs[0]["calls"] == 4


def test_cpu_threads_within_the_host_share():
    assert 1 <= bench.cpu_threads() <= 16
