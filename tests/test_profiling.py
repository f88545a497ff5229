"""Host logic of the measurement records: HBM traffic from FETCH_SIZE / WRITE_SIZE calibrated on a copy
kernel, VALU instructions per node and the held clock, and bench.py's gate on the kernel sources."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2403_13406_amd import profiling  # noqa: E402

STAGE = "void k_stage<eslb::Euler2, 2, true, false>(eslb::Grid, ...)"
COPY = "__amd_rocclr_copyBuffer"


def write_counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_scales_each_counter_by_the_copy_kernel(tmp_path):
    copy_bytes = 1 << 30
    # the copy reads 2^30 B but FETCH_SIZE reports half of it in KiB, WRITE_SIZE all of it; a smaller
    # copy dispatch (not the calibration one) must be ignored
    fetch = [(STAGE, "FETCH_SIZE", 1000.0), (STAGE, "FETCH_SIZE", 1200.0),
             (COPY, "FETCH_SIZE", copy_bytes / 2048.0), (COPY, "FETCH_SIZE", 3.0)]
    write = [(STAGE, "WRITE_SIZE", 2000.0), (STAGE, "WRITE_SIZE", 2200.0),
             (COPY, "WRITE_SIZE", copy_bytes / 1024.0), (COPY, "WRITE_SIZE", 5.0)]
    write_counters(tmp_path / "f.csv", fetch)
    write_counters(tmp_path / "w.csv", write)
    r = profiling.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_stage<eslb::Euler2", copy_bytes)
    assert r["dispatches"] == 2
    assert r["scale_fetch"] == pytest.approx(2.0) and r["scale_write"] == pytest.approx(1.0)
    assert r["bytes_per_launch"] == pytest.approx(1100.0 * 1024 * 2.0 + 2100.0 * 1024 * 1.0)


def test_valu_per_node_flops_and_clock(tmp_path):
    nodes = 64 * 1000  # 1000 waves
    rows = []
    for disp in range(2):
        rows += [(STAGE, "SQ_INSTS_VALU", 1000 * 1100.0), (STAGE, "SQ_INSTS_VALU_ADD_F64", 1000 * 100.0),
                 (STAGE, "SQ_INSTS_VALU_MUL_F64", 1000 * 300.0), (STAGE, "SQ_INSTS_VALU_FMA_F64", 1000 * 400.0),
                 (STAGE, "SQ_INSTS_VALU_TRANS_F64", 1000 * 10.0), (STAGE, "GRBM_GUI_ACTIVE", 8 * 1.7e6)]
    write_counters(tmp_path / "v.csv", rows)
    r = profiling.valu(str(tmp_path / "v.csv"), "k_stage<eslb::Euler2", nodes, kernel_us=1000.0)
    li = r["lane_instructions_per_node"]
    # wave instructions x 64 lanes / nodes: one instruction per node for every wave instruction here
    assert li["SQ_INSTS_VALU"] == pytest.approx(1100.0)
    assert r["fp64_flop_per_node"] == pytest.approx(100 + 300 + 2 * 400 + 10)
    assert r["dispatches"] == 2
    # 1.7e6 busy cycles per die over 1000 us: 1.7 GHz
    assert r["clock_ghz"] == pytest.approx(1.7)


def test_unknown_kernel_is_an_error(tmp_path):
    write_counters(tmp_path / "v.csv", [(STAGE, "SQ_INSTS_VALU", 1.0)])
    with pytest.raises(SystemExit):
        profiling.valu(str(tmp_path / "v.csv"), "k_adjoint_stage", 64)


def test_bench_uses_a_record_only_for_the_sources_it_measured(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    rec = {"bytes_per_launch": 1.0, "source_hash": profiling.source_hash()}
    with open(tmp_path / "profiles" / "traffic_x.json", "w") as fh:
        json.dump(rec, fh)
    assert bench.counter_record("traffic", "x") == rec
    rec["source_hash"] = "0" * 16
    with open(tmp_path / "profiles" / "traffic_x.json", "w") as fh:
        json.dump(rec, fh)
    assert bench.counter_record("traffic", "x") is None
    assert bench.counter_record("valu", "x") is None
