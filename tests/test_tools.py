"""Host-side tools: the rocprofv3 summary writer and the bench's one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2207_11333_amd import profile_summary as ps  # noqa: E402


def _write_counters(path, counter, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": k, "Counter_Name": counter,
                        "Counter_Value": v})


def test_traffic_scaling_by_calibration_copy(tmp_path):
    B = 1 << 20                                    # the copy moves 1 MiB each way
    # the fetch counter sees half of what the copy reads, the write counter all of it
    _write_counters(tmp_path / "f.csv", "FETCH_SIZE",
                    [("k_calib_copy(...)", B / 1024 / 2), ("k_x<1>(...)", 100.0),
                     ("k_x<1>(...)", 300.0), ("other", 7.0)])
    _write_counters(tmp_path / "w.csv", "WRITE_SIZE",
                    [("k_calib_copy(...)", B / 1024), ("k_x<1>(...)", 50.0),
                     ("k_x<1>(...)", 50.0)])
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    out = tmp_path / "t.txt"
    ps.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_x<1>", B, [str(src)],
               "title", ["cmd a", "cmd b"], str(out), algorithmic=1000.0)
    info = ps.read_summary(str(out))
    assert float(info["fetch_factor"]) == pytest.approx(2.0)
    assert float(info["write_factor"]) == pytest.approx(1.0)
    # mean of 100 and 300 KiB, doubled; 50 KiB written
    assert float(info["fetch_bytes_per_launch"]) == pytest.approx(200 * 1024 * 2)
    assert float(info["write_bytes_per_launch"]) == pytest.approx(50 * 1024)
    assert info["sources_sha256"] == ps.sources_digest([str(src)])
    src.write_text("kernel source, changed")
    assert info["sources_sha256"] != ps.sources_digest([str(src)])


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_committed_traffic_summaries_parse():
    import bench
    for name, _ in [bench.UPDATE_GEMM_TRAFFIC, *bench.AGGREGATE_TRAFFIC.values()]:
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            continue
        info = ps.read_summary(path)
        assert float(info["traffic_bytes_per_launch"]) > 0
        assert len(info["sources_sha256"]) == 64
