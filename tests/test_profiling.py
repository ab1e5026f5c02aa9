"""Host logic of the profile summaries (paper_1405_0942_amd/profiling.py) on synthetic
rocprofv3 CSV files: counter calibration on the 1 GiB copy, per-stage averages, the SQ
medians and the summary parser.  No GPU."""
import csv
import os

import pytest

from paper_1405_0942_amd import profiling as P

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
STAGE = "void relax::(anonymous namespace)::stage_kernel<{s}, false, true, {d}>(relax::SweepArgs)"


def write_run(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for disp, name, ctr, val in rows:
            r = {k: "0" for k in FIELDS}
            r.update(Dispatch_Id=str(disp), Kernel_Name=name, Counter_Name=ctr, Counter_Value=str(val))
            w.writerow(r)


def test_traffic_calibrates_on_the_copy_and_skips_diagnostics(tmp_path):
    kib = P.COPY_BYTES / 1024.0
    disp = [(1, "__amd_rocclr_copyBuffer"), (2, STAGE.format(s=4, d="false")), (3, STAGE.format(s=4, d="false")),
            (4, STAGE.format(s=1, d="true"))]
    fetch = {1: kib / 2, 2: 1000.0, 3: 1200.0, 4: 9999.0}  # FETCH_SIZE reads half the copy's bytes
    write = {1: kib, 2: 300.0, 3: 500.0, 4: 9999.0}
    write_run(tmp_path / "f", [(d, n, "FETCH_SIZE", fetch[d]) for d, n in disp])
    write_run(tmp_path / "w", [(d, n, "WRITE_SIZE", write[d]) for d, n in disp])
    per, fs, ws = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), mixed=False)
    assert fs == pytest.approx(2.0) and ws == pytest.approx(1.0)
    assert list(per) == [4]  # the diagnostics instance of stage 1 is not a stepping sweep
    assert per[4]["launches"] == 2
    assert per[4]["fetch_bytes"] == pytest.approx(1100.0 * 2 * 1024)
    assert per[4]["write_bytes"] == pytest.approx(400.0 * 1024)


def test_traffic_rejects_mismatched_runs_and_missing_copy(tmp_path):
    write_run(tmp_path / "f", [(1, STAGE.format(s=2, d="false"), "FETCH_SIZE", 1.0)])
    write_run(tmp_path / "w", [(2, STAGE.format(s=2, d="false"), "WRITE_SIZE", 1.0)])
    with pytest.raises(ValueError):
        P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), mixed=False)
    write_run(tmp_path / "w2", [(1, STAGE.format(s=2, d="false"), "WRITE_SIZE", 1.0)])
    with pytest.raises(ValueError):
        P.traffic(str(tmp_path / "f"), str(tmp_path / "w2"), mixed=False)


def test_sq_counters_take_the_median_over_launches(tmp_path):
    rows = []
    for disp, v in enumerate([5.0, 100.0, 110.0, 120.0]):  # one stage-1 launch of a retry exits at once
        rows.append((disp, STAGE.format(s=1, d="false"), "SQ_INSTS_VALU", v))
    write_run(tmp_path / "a", rows)
    write_run(tmp_path / "b", [(0, STAGE.format(s=1, d="false"), "SQ_WAVES", 2048.0)])
    per = P.sq_counters([str(tmp_path / "a"), str(tmp_path / "b")], mixed=False)
    assert per[1]["SQ_INSTS_VALU"] == 110.0 and per[1]["SQ_WAVES"] == 2048.0


def test_read_traffic_parses_committed_summaries():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for tag in ("fp64", "fp32-mixed"):
        rec = P.read_traffic(os.path.join(root, "profiles", f"stage_kernel_abc_256_{tag}_traffic.txt"))
        assert rec is not None and len(rec["source_sha256"]) == 64
        for s in range(1, 7):
            assert float(rec[f"stage{s}_bytes_per_node"]) > 0
    assert P.read_traffic(os.path.join(root, "profiles", "no_such_file.txt")) is None


def test_pipe_summary_normalises_busy_counters_and_counts(tmp_path, capsys):
    name = "void relax::(anonymous namespace)::stage_kernel<3, false, true, false, false, false>(relax::SweepArgs)"
    nodes = 64 * 1000
    rows = [(1, name, "GRBM_GUI_ACTIVE", 8 * 1000.0),   # 1000 cycles per XCD
            (1, name, "TA_TA_BUSY", 256 * 750.0),       # every TA busy 750 of them
            (1, name, "TCP_TCC_READ_REQ", 76.0 * 1000)]  # 76 requests per 64 nodes
    write_run(tmp_path / "p", rows)
    P.main(["pipe", "--run", str(tmp_path / "p"), "--workload", "w", "--precision", "fp64",
            "--nodes", str(nodes), "--command", "cmd"])
    out = capsys.readouterr().out
    row = [ln for ln in out.splitlines() if ln.startswith("| 3 |")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1:] == ["75 %", "76.0"]


def test_stage_names_of_every_sweep_variant():
    base = "void relax::(anonymous namespace)::stage_kernel<{}>(relax::SweepArgs)"
    assert P._stage_of(base.format("2, true, false")) == (2, True)
    assert P._stage_of(base.format("4, false, true, false, false, false")) == (4, False)
    assert P._stage_of(base.format("6, false, true, false, false, true")) == (6, False)  # octilateral
    assert P._stage_of(base.format("1, false, true, true, false, false")) is None       # diagnostics
    assert P._short(base.format("5, false, true, false, false, true")) == \
        "stage_kernel<5, false, true, false, false, true>"
