"""Host-side pieces of bench.py: the one-GPU guard, the rocprofv3 CSV
summary and the counter-summary reader (no GPU needed)."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id",
       "Thread_Id", "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size",
       "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
       "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp",
       "End_Timestamp"]
STAGE = ("void bssn::k_stage_lds<4>(bssn::Patch, bssn::Gauge, int, "
         "bssn::TileMap)")
F32 = ("void bssn::k_stage_lds_f32<4>(bssn::Patch, bssn::Gauge, int, "
       "bssn::TileMap)")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HDR)
        for did, name, cnt, val in rows:
            w.writerow([did, did, "Agent 1", 1, 1, 1, 256, 8, name, 256, 0, 0,
                        256, 256, 100, cnt, val, 0, 1])


def test_summary_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    f, w = tmp_path / "f", tmp_path / "w"
    f.mkdir()
    w.mkdir()
    copy = "__amd_rocclr_copyBuffer"
    _write(f / "run_counter_collection.csv",
           [(1, copy, "FETCH_SIZE", 7.0)] +
           [(2 + i, STAGE, "FETCH_SIZE", 1000.0) for i in range(4)] +
           [(10 + i, F32, "FETCH_SIZE", 900.0) for i in range(4)] +
           [(6 + i, copy, "FETCH_SIZE", 524288.0) for i in range(3)])
    _write(w / "run_counter_collection.csv",
           [(2 + i, STAGE, "WRITE_SIZE", 500.0) for i in range(4)] +
           [(10 + i, F32, "WRITE_SIZE", 400.0) for i in range(4)] +
           [(6 + i, copy, "WRITE_SIZE", 1048576.0) for i in range(3)])
    text = bench.summarize_profile([str(f), str(w)], 4)
    kv = dict(l.split(": ", 1) for l in text.splitlines()
              if not l.startswith("#"))
    assert float(kv["fetch_kib_per_launch"]) == 1000.0
    assert float(kv["mixed_f32_fetch_kib_per_launch"]) == 900.0
    assert float(kv["mixed_f32_write_kib_per_launch"]) == 400.0
    assert "mixed_f64pass_fetch_kib_per_launch" not in kv
    assert float(kv["copy_fetch_kib"]) == 524288.0   # last 3 copies only
    # FETCH reads half the copied bytes here, WRITE all of them
    assert bench.traffic_bytes(kv) == pytest.approx(2 * 1000 * 1024 +
                                                    500 * 1024)
    # a summary stamped with other sources is not used
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_k_x_w9.txt").write_text(
        text.replace(kv["source_sha256"], "0" * 16))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: kv["source_sha256"])
    got, why = bench.profile_figures("w9", "k_x")
    assert got is None and "changed" in why
    (prof / "traffic_k_x_w9.txt").write_text(text)
    got, _ = bench.profile_figures("w9", "k_x")
    assert got["write_kib_per_launch"] == "500"


def test_source_hash_ignores_comments_not_code():
    src = {f: open(os.path.join(ROOT, "paper_1111_3344_amd", "csrc", f)).read()
           for f in bench.KERNEL_SOURCES}
    h0 = bench.kernel_source_hash(src)
    assert h0 == bench.kernel_source_hash()
    f = bench.KERNEL_SOURCES[-1]
    commented = dict(src)
    commented[f] = "// a new comment\n/* and a block\n comment */\n" + \
        src[f].replace("\n", "\n  ", 3)
    assert bench.kernel_source_hash(commented) == h0
    changed = dict(src)
    changed[f] = src[f] + "\nint extra_symbol = 1;\n"
    assert bench.kernel_source_hash(changed) != h0
