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
    for name, _ in [*bench.SITE_TRAFFIC.values(), *bench.AGGREGATE_TRAFFIC.values()]:
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            continue
        info = ps.read_summary(path)
        assert float(info["traffic_bytes_per_launch"]) > 0
        assert len(info["sources_sha256"]) == 64


def test_counter_summary_derived_figures(tmp_path):
    """Per-family means and the derived MFMA / LDS figures of the counters
    mode: busy = cycles / (GUI-active per XCD x SIMDs), executed FLOPs = MOPS
    x 512, bank conflicts per conflict-free LDS cycle."""
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = []
    for d, kern in ((1, "k_a<1>(x)"), (2, "k_a<1>(x)"), (3, "k_b(y)")):
        vals = {"SQ_VALU_MFMA_BUSY_CYCLES": 1024.0 * 100 * d, "GRBM_GUI_ACTIVE": 8 * 400.0,
                "SQ_INSTS_VALU_MFMA_MOPS_F32": 10.0 * d, "SQ_LDS_BANK_CONFLICT": 25.0,
                "SQ_LDS_IDX_ACTIVE": 125.0}
        rows += [{"Dispatch_Id": d, "Kernel_Name": kern, "Counter_Name": n, "Counter_Value": v}
                 for n, v in vals.items()]
    path = tmp_path / "c.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        w.writerows(rows)
    out = tmp_path / "s.txt"
    ps.counters(str(path), ["k_a<1>", "k_b"], 1024, "t", ["cmd"], str(out), flops=[7680.0, None])
    text = out.read_text().split("kernel: ")
    a, b = text[1], text[2]
    # k_a: busy cycles mean 150 per SIMD over 400 active cycles per XCD
    assert "mfma_busy: 0.3750" in a and "dispatches: 2" in a
    assert "mfma_flops_executed: 7680" in a and "executed_over_algorithmic: 1.000" in a
    assert "lds_bank_conflict_ratio: 0.250" in a
    assert "mfma_busy: 0.7500" in b


def test_site_work_counts_the_least_work_per_launch():
    """The bench's algorithmic work per launch site: decomposed message
    linear, update linear by degree bucket (F + 4H), layer 0 with 9 real
    features, averaged over the layers."""
    import bench
    from paper_2207_11333_amd import synth
    w = synth.WORKLOADS["c1_train_fp32"]
    N, E, H, L = 4484, 9584, w.hidden, w.num_layers
    Fs = [9] + [H] * (L - 1)
    upd, per = bench.site_work("update_gemm", w, N, E)
    assert per == L and upd == pytest.approx(sum(2 * N * (F + 4 * H) * H for F in Fs) / L)
    msg, per = bench.site_work("message_gemm", w, N, E)
    assert per == L and msg == pytest.approx(sum(2 * N * F * 2 * H for F in Fs) / L)
    dh, per = bench.site_work("input_gemm", w, N, E)
    assert per == L - 1 and dh == pytest.approx(2 * N * 3 * H * H)
    w3 = synth.WORKLOADS["c3_large_bf16"]
    _, per = bench.site_work("message_gemm", w3, N, E)
    assert per == 2 * w3.num_layers          # recomputed in the backward pass
    agg, per = bench.site_work("aggregate", w, N, E)
    assert agg == pytest.approx(bench.aggregate_bytes(N, E, H, w.edge_feat))
