"""CPU tests of the rocprofv3 summaries (paper_2604_19176_amd/profiling.py) on
small synthetic CSV files shaped like rocprofv3's output."""
import csv
import os

from paper_2604_19176_amd import profiling as pr

NAME = "void pat::k_spread<4, 64>(pat::PlanDev, pat::WsLayout, pat::InstPtrs, int)"
COPY = "pat::k_stream_copy(void const*, void*, unsigned long)"


def _write(path, rows, fields):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)
    return str(path)


def _counters(path, spec):
    """spec: [(kernel, grid, counter, value)] -> a counter-collection CSV, one dispatch per row."""
    rows = [{"Dispatch_Id": i, "Kernel_Name": k, "Grid_Size": g, "Counter_Name": c, "Counter_Value": v}
            for i, (k, g, c, v) in enumerate(spec)]
    return _write(path, rows, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])


def test_short_names():
    assert pr._short(NAME) == "k_spread<4, 64>"
    assert pr._short(COPY) == "k_stream_copy"


def test_kernel_durations_per_grid(tmp_path):
    rows = [{"Kernel_Name": NAME, "Grid_Size": 64, "Start_Timestamp": 1000 * i, "End_Timestamp": 1000 * i + 500}
            for i in range(4)]
    rows += [{"Kernel_Name": NAME, "Grid_Size": 32, "Start_Timestamp": 0, "End_Timestamp": 300}]
    kd = pr.kernel_durations(_write(tmp_path / "t.csv", rows, ["Kernel_Name", "Grid_Size", "Start_Timestamp",
                                                              "End_Timestamp"]))
    assert kd[("k_spread<4, 64>", 64)] == {"n": 4, "avg_us": 0.5}
    assert kd[("k_spread<4, 64>", 32)] == {"n": 1, "avg_us": 0.3}


def test_main_grid_is_the_full_batch_launch():
    # full-batch launches (per-kernel timing), twice as many half-batch launches
    # (two-stream steps), many single-instance launches
    assert pr._main_grid({640: 10, 320: 20, 10: 50}) == 640
    # a grid seen fewer than three times (a stray call) is not the main one
    assert pr._main_grid({1280: 1, 640: 10}) == 640
    assert pr._main_grid({7: 1}) == 7


def test_traffic_scales_by_the_copy_and_picks_the_main_grid(tmp_path):
    calib = 1 << 20
    # FETCH_SIZE counts the copy's reads as half their bytes; WRITE_SIZE as all
    fetch = _counters(tmp_path / "f.csv",
                      [(COPY, 4096, "FETCH_SIZE", calib / 2048.0)] +
                      [(NAME, 640, "FETCH_SIZE", 100.0)] * 3 + [(NAME, 320, "FETCH_SIZE", 50.0)] * 6)
    write = _counters(tmp_path / "w.csv",
                      [(COPY, 4096, "WRITE_SIZE", calib / 1024.0)] +
                      [(NAME, 640, "WRITE_SIZE", 40.0)] * 3 + [(NAME, 320, "WRITE_SIZE", 20.0)] * 6)
    t = pr.traffic(fetch, write, "k_spread<4, 64>", calib)
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["fetch_bytes_per_launch"] == 100.0 * 1024 * 2.0
    assert t["write_bytes_per_launch"] == 40.0 * 1024
    assert t["dispatches"] == [3, 3]


def test_read_bytes_by_request_size(tmp_path):
    spec = []
    for d in range(3):
        spec += [(NAME, 640, "TCC_EA0_RDREQ_32B_sum", 2.0), (NAME, 640, "TCC_EA0_RDREQ_64B_sum", 1.0),
                 (NAME, 640, "TCC_EA0_RDREQ_128B_sum", 4.0), (NAME, 640, "TCC_EA0_RDREQ_sum", 7.0)]
    rows = [{"Dispatch_Id": i // 4, "Kernel_Name": k, "Grid_Size": g, "Counter_Name": c, "Counter_Value": v}
            for i, (k, g, c, v) in enumerate(spec)]
    path = _write(tmp_path / "r.csv", rows, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
                                             "Counter_Value"])
    by = pr.read_bytes_by_size(path)
    assert by[("k_spread<4, 64>", 640)] == [2 * 32 + 64 + 4 * 128.0] * 3


def test_source_hash_ignores_comments(tmp_path):
    for f in pr.KERNEL_FILES:
        (tmp_path / f).write_text("int a; // note\n/* block */ int b;\n")
    h0 = pr.source_hash(str(tmp_path))
    (tmp_path / pr.KERNEL_FILES[0]).write_text("int a;   // another note\n int b;\n")
    assert pr.source_hash(str(tmp_path)) == h0
    (tmp_path / pr.KERNEL_FILES[0]).write_text("int a; int c;\n")
    assert pr.source_hash(str(tmp_path)) != h0
    assert os.path.isdir(str(tmp_path))
