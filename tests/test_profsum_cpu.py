"""The profile summaries (paper_2307_03452_amd/profsum.py) on small synthetic
rocprofv3 CSV files: dispatch filtering by kernel and grid, the timed mean,
the copy-calibrated HBM bytes and the counter ratios."""
import csv
import json

import pytest

from paper_2307_03452_amd import profsum

TRACE_COLS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Start_Timestamp", "End_Timestamp"]
PMC_COLS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(path, cols, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(cols, r)))
    return str(path)


def test_trace_keeps_one_kernel_and_grid_and_skips_warmup(tmp_path, capsys):
    k = "void eri4::eri4_fused_kernel<2, 0>(eri4::ClassParams, double const*)"
    rows = [(1, k, 6553600, 512, 0, 1500), (2, k, 6553600, 512, 2000, 3000), (3, k, 6553600, 512, 4000, 5200),
            (4, k, 1024, 512, 6000, 9000),  # another grid: not counted
            (5, "copyBuffer", 100, 64, 9000, 9100)]
    t = _write(tmp_path / "t.csv", TRACE_COLS, rows)
    out = tmp_path / "s.md"
    profsum.main(["trace", "--csv", t, "--kernel", "eri4_fused_kernel", "--grid", "6553600", "--flops", "1.1e9",
                  "--out", str(out)])
    text = out.read_text()
    assert "3 dispatches" in text
    assert "mean 1100 ns over the 2 after the first 1" in text  # (1000 + 1200) / 2
    assert "-> 1000.00 TFLOP/s" in text  # 1.1e9 flops / 1.1 us
    assert "eri4_fused_kernel<2, 0>" in text and "copyBuffer x1" in text
    assert "eri4::eri4_fused_kernel<2, 0> x1" in text  # the other grid, listed as not counted


def test_traffic_divides_by_the_copy_calibration(tmp_path, capsys):
    k = "eri4_fused_kernel<2, 0>"
    f = _write(tmp_path / "f.csv", PMC_COLS, [(1, k, 64, "FETCH_SIZE", 100.0), (2, k, 64, "FETCH_SIZE", 300.0),
                                               (3, k, 32, "FETCH_SIZE", 9999.0)])
    w = _write(tmp_path / "w.csv", PMC_COLS, [(1, k, 64, "WRITE_SIZE", 400.0)])
    cf = _write(tmp_path / "cf.csv", PMC_COLS, [(1, "add_kernel", 8, "FETCH_SIZE", 512.0)])  # 0.5 of 1 MiB read
    cw = _write(tmp_path / "cw.csv", PMC_COLS, [(1, "add_kernel", 8, "WRITE_SIZE", 1024.0)])  # 1.0 of 1 MiB
    out = tmp_path / "t.json"
    profsum.main(["traffic", "--fetch", f, "--write", w, "--copy-fetch", cf, "--copy-write", cw, "--kernel",
                  "eri4_fused_kernel", "--grid", "64", "--copy-kernel", "add", "--copy-bytes", str(1 << 20),
                  "--algorithmic-bytes", str(800 * 1024), "--out", str(out)])
    d = json.loads(out.read_text())
    assert d["fetch_size_kib_per_dispatch"] == pytest.approx(200.0)
    assert d["copy_calibration"]["fetch_factor"] == pytest.approx(0.5)
    assert d["copy_calibration"]["write_factor"] == pytest.approx(1.0)
    assert d["hbm_bytes_per_launch"] == pytest.approx(200 * 1024 / 0.5 + 400 * 1024)
    assert d["traffic_over_algorithmic"] == pytest.approx(1.0)


def test_counters_ratios(tmp_path, capsys):
    k = "eri4_fused_kernel<2, 0>"
    a = _write(tmp_path / "a.csv", PMC_COLS, [
        (1, k, 64, "GRBM_GUI_ACTIVE", 8.0e6), (1, k, 64, "SQ_VALU_MFMA_BUSY_CYCLES", 5.12e8),
        (1, k, 64, "SQ_INSTS_MFMA", 8.0e6), (1, k, 64, "SQ_WAVE_CYCLES", 1.0e6),
        (2, k, 128, "SQ_INSTS_MFMA", 1.0), (1, "other", 64, "SQ_INSTS_MFMA", 1.0)])
    b = _write(tmp_path / "b.csv", PMC_COLS, [
        (1, k, 64, "GRBM_GUI_ACTIVE", 8.0e6), (1, k, 64, "SQ_WAIT_INST_ANY", 2.5e5),
        (1, k, 64, "SQ_LDS_BANK_CONFLICT", 2.56e7), (1, k, 64, "SQ_ACTIVE_INST_LDS", 100.0)])
    out = tmp_path / "c.md"
    profsum.main(["counters", "--csv", a, b, "--kernel", "eri4_fused_kernel", "--grid", "64", "--duration-ns",
                  "1e6", "--out", str(out)])
    text = out.read_text()
    # 8e6 / 8 XCDs = 1e6 kernel cycles; 1024 SIMDs -> 1.024e9 SIMD cycles
    assert "| SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x kernel cycles) | 0.500 |" in text
    assert "| SQ_INSTS_MFMA x 64 cycles / (1024 SIMDs x kernel cycles) | 0.500 |" in text
    assert "(waves waiting on any dependency) | 0.250 |" in text
    assert "| SQ_LDS_BANK_CONFLICT / (256 CUs x kernel cycles) (share of LDS cycles lost to bank conflicts) | 0.100 |" in text
    assert "1.000 GHz" in text
    assert "| GRBM_GUI_ACTIVE | 8e+06 | 2 |" in text  # one dispatch from each pass


def test_counters_select(tmp_path, capsys):
    k = "eri4_small_kernel<3, 3>"
    a = _write(tmp_path / "a.csv", PMC_COLS, [(i, k, 64, "SQ_INSTS_MFMA", float(i)) for i in range(6)])
    out = tmp_path / "c.md"
    profsum.main(["counters", "--csv", a, "--kernel", "eri4_small_kernel", "--grid", "64", "--select", "2:5",
                  "--out", str(out)])
    assert "| SQ_INSTS_MFMA | 3 | 3 |" in out.read_text()  # mean of 2, 3, 4
