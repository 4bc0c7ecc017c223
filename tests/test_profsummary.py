"""Host logic of the rocprofv3 summaries: the copy-probe window of the HBM byte counters."""
import csv
import os

from paper_0901_3512_amd.profsummary import _copy_window, bytes_per_launch


def _row(d, k, v, name):
    return {"Dispatch_Id": str(d), "Kernel_Name": k, "Counter_Value": str(v), "Counter_Name": name}


def test_probe_is_the_first_run_of_big_copies():
    rows = [_row(1, "copyBuffer", 10, "X"), _row(2, "hop_a", 5, "X"), _row(3, "copyBuffer", 1000, "X"),
            _row(4, "copyBuffer", 990, "X"), _row(5, "copyBuffer", 1010, "X"), _row(6, "hop_a", 7, "X"),
            _row(7, "hop_a", 9, "X"), _row(8, "copyBuffer", 1000, "X"), _row(9, "hop_a", 3, "X")]
    ref, last, nxt = _copy_window(rows)
    assert ref == 1000.0 and last == 5 and nxt == 8


def test_probe_is_found_beside_larger_single_copies():
    # a basis growing by device copies (single, larger copies) before and after the probe's run
    rows = [_row(1, "copyBuffer", 5000, "X"), _row(2, "hop_a", 5, "X"), _row(3, "copyBuffer", 1000, "X"),
            _row(4, "copyBuffer", 1000, "X"), _row(5, "copyBuffer", 1000, "X"), _row(6, "hop_a", 7, "X"),
            _row(7, "copyBuffer", 9000, "X"), _row(8, "hop_a", 9, "X"), _row(9, "copyBuffer", 1000, "X")]
    ref, last, nxt = _copy_window(rows)
    assert ref == 1000.0 and last == 5 and nxt == 9


def test_probe_is_found_after_smaller_runs_of_copies():
    # a batch placing its same-shape configurations by back-to-back device copies before the probe
    rows = [_row(1, "copyBuffer", 20, "X"), _row(2, "copyBuffer", 20, "X"), _row(3, "copyBuffer", 21, "X"),
            _row(4, "hop_a", 5, "X"), _row(5, "copyBuffer", 1000, "X"), _row(6, "copyBuffer", 1000, "X"),
            _row(7, "copyBuffer", 1000, "X"), _row(8, "hop_a", 7, "X"), _row(9, "copyBuffer", 1000, "X"),
            _row(10, "copyBuffer", 1000, "X")]
    ref, last, nxt = _copy_window(rows)
    assert ref == 1000.0 and last == 7 and nxt == 9


def _write(d, name, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow({**r, "Counter_Name": name})


def test_bytes_per_launch_counts_only_the_timed_window(tmp_path):
    # the probe reads 524,288 KiB for a 1 GiB copy (scale 2) and writes 1,048,576 KiB (scale 1)
    fetch = [_row(1, "hop_a", 999, ""), _row(2, "copyBuffer", 524288, ""), _row(3, "hop_a", 100, ""),
             _row(4, "hop_a", 300, ""), _row(5, "copyBuffer", 524288, ""), _row(6, "hop_a", 999, "")]
    write = [_row(1, "hop_a", 999, ""), _row(2, "copyBuffer", 1048576, ""), _row(3, "hop_a", 50, ""),
             _row(4, "hop_a", 50, ""), _row(5, "copyBuffer", 1048576, ""), _row(6, "hop_a", 999, "")]
    _write(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write(str(tmp_path / "w"), "WRITE_SIZE", write)
    r = bytes_per_launch(str(tmp_path / "f"), str(tmp_path / "w"), "hop_")
    assert r["dispatches"] == 2
    assert r["fetch_bytes"] == 200 * 2.0 * 1024 and r["write_bytes"] == 50 * 1.0 * 1024


def test_counters_derive_mfma_busy_fraction_and_rate(tmp_path):
    from paper_0901_3512_amd.profsummary import counters
    d = tmp_path / "m"
    d.mkdir()
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
                                          "End_Timestamp"])
        w.writeheader()
        for dsp in (1, 2):
            for cn, v in (("SQ_INSTS_VALU_MFMA_MOPS_F64", 1e6), ("GRBM_GUI_ACTIVE", 8e6),
                          ("SQ_VALU_MFMA_BUSY_CYCLES", 1024e6 * 0.25)):
                w.writerow(dict(Dispatch_Id=dsp, Kernel_Name="void scg::proj_kernel<double, double>(a)", Counter_Name=cn,
                                Counter_Value=v, Start_Timestamp=0, End_Timestamp=1000000))
            w.writerow(dict(Dispatch_Id=10 + dsp, Kernel_Name="void scg::other(a)", Counter_Name="GRBM_GUI_ACTIVE",
                            Counter_Value=1, Start_Timestamp=0, End_Timestamp=1))
    out = counters(str(d), "proj_kernel")
    assert "dispatches 2" in out and "MFMA busy fraction 0.2500" in out and "F64 TFLOP/s 0.51" in out
    assert "other" not in out
