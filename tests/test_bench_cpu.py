"""Host logic of bench.py (CPU only): kernel names, the algorithmic-byte count, the
rocprofv3 summaries behind the roofline object, and the one-GPU contract."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SEARCH = "void gm::(anonymous namespace)::search_kernel<{}, {}, {}, {}, {}>(gm::SearchArgs)"


def test_kernel_keys():
    assert bench.kernel_key(SEARCH.format(0, "true", "false", "false", 4)) == "search<slim>"
    assert bench.kernel_key(SEARCH.format(0, "true", "false", "false", 5)) == "search<slim,5w>"
    assert bench.kernel_key(SEARCH.format(1, "true", "true", "true", 4)) == "enumerate<slim,sb,cg>"
    assert bench.kernel_key(SEARCH.format(2, "false", "true", "false", 4)) == "expand<full,sb>"
    assert bench.kernel_key("__amd_rocclr_copyBuffer") == "copy"
    assert bench.kernel_key("gm::(anonymous namespace)::cand_fill_kernel(int const*)") == "cand_fill_kernel"


def test_traffic_summary_is_used_only_for_the_same_sources(tmp_path):
    f = tmp_path / "traffic.txt"
    f.write_text(f"# header\n\nkernel_sha: {bench.kernel_sha()}\ntraffic_bytes_per_launch: 12345\n")
    assert bench.read_traffic(str(f)) == {"bytes_per_launch": 12345.0}
    f.write_text("kernel_sha: 0000000000000000\ntraffic_bytes_per_launch: 12345\n")
    assert bench.read_traffic(str(f)) is None
    assert bench.read_traffic(str(tmp_path / "missing.txt")) is None
    assert bench.traffic_file_for("rmat24_ef16_zipf8_q12-32").endswith("profiles/search_kernel_rmat24_q12-32_traffic.txt")


def test_roofline_uses_the_issued_bytes():
    class R:
        def __init__(self, ms, b, late):
            self.kernel_ms, self.kernel_bytes, self.kernel_bytes_late = ms, b, late
    rf = bench.roofline([R(2.0, 8e9, 1e9), R(2.0, 8e9, 0.0)], "/nonexistent")
    assert rf["launches"] == 2 and rf["avg_launch_ms"] == 2.0
    assert rf["achieved"] == 4000.0 and rf["frac"] == 0.5
    assert rf["issued_bytes_per_launch"] == 8e9 and rf["late_bytes_per_launch_max"] == 0.5e9
    assert abs(rf["frac_excluding_late"] - 0.46875) < 1e-12
    assert rf["traffic"] is None


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_stats_and_counter_summaries(tmp_path):
    stats = tmp_path / "stats" / "run_kernel_stats.csv"
    _write_csv(str(stats), ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs", "Percentage"],
               [[SEARCH.format(0, "true", "false", "false", 5), 2, 6e6, 3e6, 2e6, 4e6, 99.0],
                ["__amd_rocclr_copyBuffer", 4, 4e3, 1e3, 1e3, 1e3, 1.0]])
    out = bench.summarize_stats(str(tmp_path / "stats"))
    assert out.splitlines()[0].startswith("search<slim,5w>")
    assert "avg_ms=   3.0000" in out.splitlines()[0] and "calls=    2" in out.splitlines()[0]

    def pmc(d, counter, search_vals, copy_vals):
        rows = [[SEARCH.format(0, "true", "false", "false", 5), counter, v] for v in search_vals]
        rows += [["__amd_rocclr_copyBuffer", counter, v] for v in copy_vals]
        _write_csv(str(tmp_path / d / "run_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
                   rows)

    # the calibration copy moves 256 MiB: FETCH_SIZE reads half of it, WRITE_SIZE all of it
    pmc("fetch", "FETCH_SIZE", [900.0, 1100.0], [131072.0, 4.0])
    pmc("write", "WRITE_SIZE", [10.0, 30.0], [262144.0])
    got = bench.pmc_per_kernel(str(tmp_path / "fetch"), "FETCH_SIZE")
    assert got["search<slim,5w>"] == (1000.0, 2) and got["copy"] == (131072.0, 1)
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-traffic",
                          str(tmp_path / "fetch"), str(tmp_path / "write"), "--copy-bytes", str(256 << 20)],
                         capture_output=True, text=True, check=True)
    kv = dict(line.split(": ", 1) for line in res.stdout.splitlines())
    assert kv["kernel"] == "search<slim,5w>"
    assert bench.merge_means([(1000.0, 2), (4000.0, 1)]) == (2000.0, 3)
    assert float(kv["fetch_scale"]) == pytest.approx(2.0) and float(kv["write_scale"]) == pytest.approx(1.0)
    assert int(kv["traffic_bytes_per_launch"]) == 1000 * 1024 * 2 + 20 * 1024


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True)
    assert res.returncode == 2
    assert "exactly one GPU" in res.stderr


def test_counter_summary_of_the_search_kernel(tmp_path):
    rows = []
    for d, (waves, cycles, wait, valu) in enumerate([(100, 1000, 600, 5000), (300, 3000, 1500, 15000)]):
        for name, v in (("SQ_WAVES", waves), ("SQ_WAVE_CYCLES", cycles), ("SQ_WAIT_ANY", wait),
                        ("SQ_INSTS_VALU", valu)):
            rows.append([d, SEARCH.format(0, "true", "false", "false", 4), name, v])
        rows.append([d, "__amd_rocclr_copyBuffer", "SQ_WAVES", 7])
    _write_csv(str(tmp_path / "pmc" / "run_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    kv = dict(line.split(": ", 1) for line in bench.summarize_pmc(str(tmp_path / "pmc")).splitlines())
    assert kv["kernel"] == "search<slim>"
    assert kv["SQ_WAVES"].startswith("400") and "(dispatches 2)" in kv["SQ_WAVES"]
    assert float(kv["wait_any_fraction"]) == 0.525   # (600 + 1500) / (1000 + 3000)
    assert kv["sq_insts_valu_per_wave"] == "50"


def test_trace_window_summary(tmp_path):
    """The timed window of a kernel trace: search dispatches in dispatch order, skip then take."""
    rows = []
    for i in range(6):  # dispatch ids out of order in the file; copies are not search dispatches
        d = [5, 0, 3, 1, 4, 2][i]
        rows.append([d, SEARCH.format(0, "true", "false", "false", 4 if d % 2 else 5), 0, (d + 1) * 1e6])
    rows.append([9, "__amd_rocclr_copyBuffer", 0, 5e6])
    _write_csv(str(tmp_path / "trace" / "run_kernel_trace.csv"),
               ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = bench.summarize_trace(str(tmp_path / "trace"), 2, 3).splitlines()
    assert out[0] == "search dispatches: 6"
    assert out[1].startswith("all: dispatches=6 avg_ms=3.5000")
    # window: dispatches 2, 3, 4 -> 3, 4, 5 ms
    assert out[2].startswith("window [2, 5): dispatches=3 avg_ms=4.0000")
    assert "search<slim,5w>: n=2 avg_ms=4.0000" in out[2] and "search<slim>: n=1 avg_ms=4.0000" in out[2]
