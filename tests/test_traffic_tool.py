"""The measurement tool behind the bench's traffic figure and the kernel-trace
summaries (paper_1611_04959_amd/traffic.py), on synthetic rocprofv3 CSV files:
counter values are scaled by the copy calibration and taken per kernel as the
median dispatch, and the last launches of a trace are found and timed."""
import csv
import json
import os

from paper_1611_04959_amd import traffic

COUNTER_FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
TRACE_FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=COUNTER_FIELDS)
        w.writeheader()
        for disp, name, value in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_summarize_scales_by_the_copy_and_takes_medians(tmp_path):
    mib = 64
    # the copy of 64 MiB reads FETCH_SIZE of about half its bytes in KiB (a factor near 2, as
    # measured on the device) and writes all of them
    write_counters(tmp_path / "cf", "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", mib * 1024 / 2 + 1)])
    write_counters(tmp_path / "cw", "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", mib * 1024)])
    # three dispatches of the scan (median 1000 KiB), one of each other pass; the
    # counter of one dispatch may come split over rows (summed)
    write_counters(tmp_path / "f", "FETCH_SIZE", [
        (10, "void daqk::(anonymous namespace)::k_scan_pass<512, 6, false, true>(daqk::KArgs)", 900.0),
        (11, "void daqk::(anonymous namespace)::k_scan_pass<512, 6, false, true>(daqk::KArgs)", 600.0),
        (11, "void daqk::(anonymous namespace)::k_scan_pass<512, 6, false, true>(daqk::KArgs)", 400.0),
        (12, "void daqk::(anonymous namespace)::k_scan_pass<512, 6, false, true>(daqk::KArgs)", 5000.0),
        (13, "void daqk::(anonymous namespace)::k_edge_pass<512>(daqk::KArgs)", 10.0),
        (14, "void daqk::(anonymous namespace)::k_copy_pass<512>(daqk::KArgs)", 300.0),
        (15, "at::native::vectorized_elementwise_kernel<4>", 77.0)])
    write_counters(tmp_path / "w", "WRITE_SIZE", [
        (10, "void daqk::(anonymous namespace)::k_scan_pass<512, 6, false, true>(daqk::KArgs)", 2.0),
        (13, "void daqk::(anonymous namespace)::k_edge_pass<512>(daqk::KArgs)", 1.0),
        (14, "void daqk::(anonymous namespace)::k_copy_pass<512>(daqk::KArgs)", 200.0)])
    out = tmp_path / "t.json"
    res = traffic.summarize(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                            str(out), fills=16, mib=mib)
    k = res["kernels"]
    assert set(k) == {"k_scan_pass", "k_edge_pass", "k_copy_pass"}
    f_fac = mib * 1024 / (mib * 1024 / 2 + 1)
    assert abs(res["copy_factor_fetch"] - f_fac) < 1e-12 and res["copy_factor_write"] == 1.0
    assert k["k_scan_pass"]["fetch_kib_raw"] == 1000.0 and k["k_scan_pass"]["dispatches"] == 3
    assert abs(k["k_scan_pass"]["fetch_bytes"] - 1000.0 * 1024 * f_fac) < 1e-6
    assert k["k_copy_pass"]["write_bytes"] == 200.0 * 1024
    total = sum(v["fetch_bytes"] + v["write_bytes"] for v in k.values())
    assert res["bytes_per_launch"] == round(total)
    assert json.load(open(out))["kernel_sha"] == traffic.kernel_sha()


def test_tail_finds_the_last_launches(tmp_path, capsys):
    path = tmp_path / "trace.csv"
    rows = [("void (anonymous namespace)::k_read_tiles<0>(short const*)", 0, 100)]
    t = 1000
    for _ in range(5):  # five launches: scan 150, edge 10, copy 70, no gaps
        for name, d in (("void daqk::(anonymous namespace)::k_scan_pass<512, 6, false, true>(daqk::KArgs)", 150),
                        ("void daqk::(anonymous namespace)::k_edge_pass<512>(daqk::KArgs)", 10),
                        ("void daqk::(anonymous namespace)::k_copy_pass<512>(daqk::KArgs)", 70)):
            rows.append((name, t * 1000, (t + d) * 1000))
            t += d
        t += 5
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(TRACE_FIELDS)
        w.writerows(rows)
    traffic.tail(str(path), 3)
    out = capsys.readouterr().out
    assert "| `k_scan_pass<512, 6, false, true>` | 3 | 150.0 |" in out
    assert "| `k_edge_pass<512>` | 3 | 10.0 |" in out
    assert "| `k_copy_pass<512>` | 3 | 70.0 |" in out
    assert "last 3 launches (first kernel start to last kernel end): 230.0 us" in out


def test_streams_measures_span_and_overlap(tmp_path, capsys):
    """Two streams, launches of 100 us offset by 50 us: four launches span
    250 us (62.5 us each), and kernels of both streams run at once for the
    150 us between the second launch's start and the third's end."""
    path = tmp_path / "trace.csv"
    rows = []
    for i in range(4):
        t = 1000 + 50 * i
        sid = str(i % 2)
        for name, a, b in (("k_scan_pass<512, 9, false, true>", 0, 60), ("k_edge_pass<512>", 60, 70),
                           ("k_copy_pass<512>", 70, 100)):
            rows.append({"Kernel_Name": "void daqk::(anonymous namespace)::%s(daqk::KArgs)" % name,
                         "Start_Timestamp": (t + a) * 1000, "End_Timestamp": (t + b) * 1000, "Stream_Id": sid})
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=TRACE_FIELDS + ["Stream_Id"])
        w.writeheader()
        w.writerows(rows)
    res = traffic.streams(str(path), 4)
    out = capsys.readouterr().out
    assert res["streams"] == {"0": 2, "1": 2}
    assert abs(res["span_us"] - 250.0) < 1e-9 and abs(res["per_launch_us"] - 62.5) < 1e-9
    assert abs(res["overlap"] - 150.0 / 250.0) < 1e-9
    assert "| `k_scan_pass` | 4 | 60.0 |" in out
