"""The measurement helpers of bench.py on synthetic rocprofv3 output (CPU):
the counter calibration and scaling, the kernel-trace summary, the
algorithmic byte counts and the stale-counter rule."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

WALK = "void ivf::(anonymous namespace)::k_walk<0>(ivf::WalkArgs)"
BATCH = "void ivf::(anonymous namespace)::k_walk_batch<0>(ivf::WalkArgs const*, long const*, int, int, unsigned long long*)"
IVFD = "void ivf::(anonymous namespace)::k_ivfd_walk<4>(ivf::IvfdArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _counter_csv(path, counter, rows):
    _write(path, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
           [{"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v}
            for i, (k, v) in enumerate(rows)])


def test_counter_scaling_uses_the_copy_calibration_and_the_last_launch(tmp_path):
    kib = bench.COPY_BYTES / 1024.0
    # the copy reads half of its bytes by this counter and writes all of them
    _counter_csv(tmp_path / "fetch.csv", "FETCH_SIZE",
                 [(COPY, kib / 2), (COPY, kib / 2), (COPY, kib / 2), (BATCH, 9e9), (WALK, 1000.0),
                  (WALK, 2000.0)])
    _counter_csv(tmp_path / "write.csv", "WRITE_SIZE",
                 [(COPY, kib), (COPY, kib), (COPY, kib), (WALK, 10.0), (WALK, 30.0)])
    out = bench.summarize_counters(str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"),
                                   "w", "f32", str(tmp_path / "t.json"), "cmd")
    assert out["fetch_scale"] == pytest.approx(2.0) and out["write_scale"] == pytest.approx(1.0)
    # the last k_walk launch (not k_walk_batch, not the copies), scaled
    assert out["fetch_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert out["write_bytes"] == pytest.approx(30.0 * 1024)
    assert out["hbm_bytes_per_launch"] == pytest.approx(out["fetch_bytes"] + out["write_bytes"])
    assert out["kernel_hash"] == bench.kernel_hash()
    assert json.load(open(tmp_path / "t.json"))["hbm_bytes_per_launch"] == out["hbm_bytes_per_launch"]


def test_counter_summary_of_the_ivfd_kernel_hashes_its_own_source(tmp_path):
    kib = bench.COPY_BYTES / 1024.0
    _counter_csv(tmp_path / "fetch.csv", "FETCH_SIZE", [(COPY, kib / 2)] * 3 + [(WALK, 5.0), (IVFD, 7.0)])
    _counter_csv(tmp_path / "write.csv", "WRITE_SIZE", [(COPY, kib)] * 3 + [(IVFD, 1.0)])
    out = bench.summarize_counters(str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"),
                                   "w", "f32", str(tmp_path / "t.json"), "cmd", "k_ivfd_walk")
    assert out["fetch_bytes"] == pytest.approx(7.0 * 1024 * 2.0)
    assert out["kernel_hash"] == bench.kernel_hash(("ivfd.hip",)) != bench.kernel_hash()


def test_trace_summary_lists_launches_and_the_steady_state_average(tmp_path):
    stats = tmp_path / "x_kernel_stats.csv"
    trace = tmp_path / "x_kernel_trace.csv"
    _write(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [{"Name": WALK, "Calls": 3, "TotalDurationNs": 2.5e9, "AverageNs": 8.3e8, "Percentage": 90},
            {"Name": "ivf::(anonymous namespace)::k_merge(ivf::MergeArgs)", "Calls": 3,
             "TotalDurationNs": 1e7, "AverageNs": 3.3e6, "Percentage": 1}])
    launches = [(0, 500_000_000), (1_000_000_000, 1_900_000_000), (2_000_000_000, 2_910_000_000)]
    _write(trace, ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "VGPR_Count",
                   "Accum_VGPR_Count", "SGPR_Count", "LDS_Block_Size", "Workgroup_Size_X",
                   "Grid_Size_X"],
           [{"Kernel_Name": WALK, "Start_Timestamp": a, "End_Timestamp": b, "VGPR_Count": 40,
             "Accum_VGPR_Count": 0, "SGPR_Count": 112, "LDS_Block_Size": 0,
             "Workgroup_Size_X": 512, "Grid_Size_X": 393216} for a, b in launches])
    out = tmp_path / "s.txt"
    bench.summarize_trace(str(stats), str(out), "the command", "a note")
    text = out.read_text()
    assert "# command: the command" in text and "# a note" in text
    assert "500.000, 900.000, 910.000" in text
    assert "after the first" in text and "905.000 ms" in text
    assert text.index("k_walk<0>") < text.index("k_merge")


def test_algorithmic_bytes_and_the_stale_counter_rule(tmp_path, monkeypatch):
    # 8 B per FP32 posting entry (id + value), 4 B for 16-bit values; per
    # cluster range: 16 B per object nonzero (id, value, 8-byte slice descriptor),
    # 8 B per row pointer, 16 B per range record written
    assert bench.walk_bytes(10, 3, 2, 1, "f32") == 80 + 48 + 24 + 32
    assert bench.walk_bytes(10, 3, 2, 4, "bf16") == 40 + 4 * (48 + 24 + 32)
    assert (bench.iteration_bytes(10, 3, 2, 1, 5, "f32")
            == bench.walk_bytes(10, 3, 2, 1, "f32") + 16 + 48 + 5 * 32)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "kernel_hash", lambda sources=("assign.hip", "invfile.hip"): "abc")
    p = tmp_path / "profiles" / "walk_w_f32_levels.json"
    p.write_text(json.dumps({"kernel_hash": "abc", "l2_read_bytes": 123.0}))
    assert bench.level_counters("k_walk", "w", "f32")["l2_read_bytes"] == 123.0
    p.write_text(json.dumps({"kernel_hash": "old", "l2_read_bytes": 123.0}))
    assert bench.level_counters("k_walk", "w", "f32") is None     # counters of another kernel
    assert bench.level_counters("k_walk", "w", "bf16") is None    # none taken


PROBE = "ivf::(anonymous namespace)::k_read(uint4 const*, long, long, long, int, int, uint4*)"


def test_level_summary_scales_requests_by_the_probes(tmp_path, monkeypatch):
    """Requests are turned into bytes by what the same counter reads for the
    timed probe of known size; the walk's last dispatch is the one used."""
    cus = 4
    l2 = bench.probe_bytes("l2", cus)
    hbm = bench.probe_bytes("hbm", cus)
    rows = []
    did = 0
    # probes: (warm, timed) per level; 128-byte L1->L2 requests, 64-byte fabric ones
    for level in bench.CEILINGS:
        for _ in range(2 * len(bench.PROBE_SHAPES)):
            nb = bench.probe_bytes(level, cus)
            for name, v in (("TCP_TCC_READ_REQ_sum", nb / 128), ("TCC_EA0_RDREQ_sum", nb / 64),
                            ("TCC_HIT_sum", 1.0), ("TCC_MISS_sum", 1.0)):
                rows.append({"Dispatch_Id": did, "Kernel_Name": PROBE, "Counter_Name": name,
                             "Counter_Value": v})
            did += 1
    for walk_req in (10.0, 1000.0):        # two walk launches: the last one counts
        for name, v in (("TCP_TCC_READ_REQ_sum", walk_req), ("TCC_EA0_RDREQ_sum", walk_req / 4),
                        ("TCC_HIT_sum", 3.0), ("TCC_MISS_sum", 1.0)):
            rows.append({"Dispatch_Id": did, "Kernel_Name": WALK, "Counter_Name": name,
                         "Counter_Value": v})
        did += 1
    _write(tmp_path / "p.csv", ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
           rows)
    out = bench.summarize_levels("w", "f32", str(tmp_path / "l.json"), str(tmp_path / "l.txt"),
                                 "cmd", "k_walk", cus, str(tmp_path / "p.csv"))
    assert out["l2_bytes_per_request"] == pytest.approx(128.0)
    assert out["fabric_bytes_per_request"] == pytest.approx(64.0)
    assert out["l2_read_bytes"] == pytest.approx(1000.0 * 128)
    assert out["fabric_read_bytes"] == pytest.approx(250.0 * 64)
    assert out["l2_hit_rate"] == pytest.approx(0.75)
    assert l2 < hbm
    # the roofline then divides by the walk time and the measured ceilings
    monkeypatch.setattr(bench, "level_counters", lambda *a: out)
    r = bench.walk_roofline("k_walk", "w", "f32", 2.0, 1e6, {"l2": 1e-4, "infinity_cache": 1e-4,
                                                             "hbm": 1e-4}, 1.0, 1.0)
    assert r["bound"] == "l2" and r["frac"] == pytest.approx(1000.0 * 128 / 2.0 / 1e9 / 1e-4)
    assert r["effective_gbps_algorithmic"] == pytest.approx(1e6 / 2.0 / 1e9)


def test_update_trace_summary_splits_iterations_at_the_walk(tmp_path):
    """Kernels after walk launch i are iteration i's; the assignment side's
    merge is listed apart from the update's busy time."""
    merge = "ivf::(anonymous namespace)::k_merge(ivf::MergeArgs)"
    keys = "ivf::(anonymous namespace)::k_keys(int const*, int const*, long, int, unsigned int*)"
    fill = "ivf::(anonymous namespace)::k_fill(ivf::UpdateArgs, long)"
    seq = [("gen", 0, 5), (WALK, 10, 100), (merge, 100, 103), (keys, 103, 107), (fill, 107, 108),
           (COPY, 108, 200), (WALK, 200, 300), (merge, 300, 303), (fill, 303, 305)]
    ns = 1_000_000
    _write(tmp_path / "t.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [{"Kernel_Name": n, "Start_Timestamp": a * ns, "End_Timestamp": b * ns}
            for n, a, b in reversed(seq)])   # any order: sorted by start
    bench.summarize_update_trace(str(tmp_path / "t.csv"), str(tmp_path / "u.txt"), "cmd")
    text = (tmp_path / "u.txt").read_text()
    assert "# command: cmd" in text
    assert "iteration 1: update busy 5.00 ms" in text
    assert "iteration 2: update busy 2.00 ms" in text
    assert "k_merge" not in text and "copyBuffer" not in text and "gen" not in text
    first = text[text.index("iteration 1"):text.index("iteration 2")]
    assert first.index("k_keys") < first.index("k_fill")


def test_trace_summary_refuses_a_trace_of_another_run(tmp_path):
    stats = tmp_path / "x_kernel_stats.csv"
    _write(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [{"Name": WALK, "Calls": 1, "TotalDurationNs": 1e9, "AverageNs": 1e9, "Percentage": 100}])
    _write(tmp_path / "x_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [{"Kernel_Name": IVFD, "Start_Timestamp": 0, "End_Timestamp": 5}])
    with pytest.raises(ValueError, match="no launch"):
        bench.summarize_trace(str(stats), str(tmp_path / "s.txt"), "cmd")
