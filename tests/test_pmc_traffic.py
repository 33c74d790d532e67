"""Host logic of the HBM-traffic tool: counter csv parsing and the copy calibration."""
import csv
import json
import os

import pytest

from paper_2108_08845_amd import pmc_traffic as pt

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_run(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, vals) in enumerate(rows):
            for v in vals:   # several values for one dispatch are summed
                w.writerow({k: "" for k in FIELDS} | {"Dispatch_Id": str(i), "Kernel_Name": name,
                                                      "Counter_Name": counter, "Counter_Value": str(v)})


def test_traffic_from_counters(tmp_path):
    k = "void psvd::k_sketch_bf16<32, 10>(psvd::FusedArgs)"
    write_run(tmp_path / "f", "FETCH_SIZE", [(k, [600.0, 400.0]), (k, [1000.0]), ("other", [5.0])])
    write_run(tmp_path / "w", "WRITE_SIZE", [(k, [10.0]), (k, [30.0])])
    # the copy counters read 2x / 0.5x the true 1 GiB
    write_run(tmp_path / "cf", "FETCH_SIZE", [("copyBuffer", [2 * 1048576.0]), ("tiny", [1.0])])
    write_run(tmp_path / "cw", "WRITE_SIZE", [("copyBuffer", [0.5 * 1048576.0])])
    rec = pt.compute(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                     "k_sketch_bf16", "fused_bf16", "wl")
    assert rec["fetch_kib_per_dispatch"] == pytest.approx(1000.0)
    assert rec["write_kib_per_dispatch"] == pytest.approx(20.0)
    assert rec["factor_fetch"] == pytest.approx(0.5) and rec["factor_write"] == pytest.approx(2.0)
    assert rec["traffic_bytes_per_launch"] == pytest.approx(1000 * 1024 * 0.5 + 20 * 1024 * 2.0)
    assert rec["source_sha256"] == pt.source_sha256("fused_bf16")
    out = tmp_path / "p"
    out.mkdir()
    (out / "t.json").write_text(json.dumps(rec))
    assert pt.load_current(str(out), "fused_bf16", "wl")["traffic_bytes_per_launch"] == rec["traffic_bytes_per_launch"]
    rec["source_sha256"] = "0" * 64   # kernel changed since the counters were taken
    (out / "t.json").write_text(json.dumps(rec))
    assert pt.load_current(str(out), "fused_bf16", "wl") is None


def test_missing_kernel_is_an_error(tmp_path):
    write_run(tmp_path / "f", "FETCH_SIZE", [("a", [1.0])])
    with pytest.raises(KeyError):
        pt.pick(pt.read_counters(str(tmp_path / "f"), "FETCH_SIZE"), "k_fused")
