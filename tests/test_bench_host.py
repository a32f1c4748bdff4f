"""Host logic of the measurement (CPU, no GPU): the roofline object bench.py
reports, the traffic figure it takes from profiles/traffic.json (dropped once
the kernel's source changes), and the rocprofv3 summaries of
paper_1609_03986_amd.profile_summary (kernel names, per-launch grouping and
the copy calibration), on synthetic counter files."""
import csv
import hashlib
import json
import os

import pytest

import bench
from paper_1609_03986_amd import profile_summary as ps


def kernels(**ms):
    return {k: {"launches_per_step": 1.0, "avg_ms": v, "ms_per_step": v} for k, v in ms.items()}


def test_roofline_takes_the_dominant_kernel_and_its_own_peak():
    r = bench.roofline_of(kernels(extract=3.0, knn_batch_fp4=4.0), 1_280_000, 25_200_000_000,
                          "nowhere")
    assert r["kernel"] == "knn_batch_fp4" and r["bound"] == "mfma"
    assert r["peak"] == 10100.0
    assert r["achieved"] == pytest.approx(25.2e9 * 1024 / 4.0e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 10100.0)
    assert r["traffic"] is None                   # no record for this workload
    e = bench.roofline_of(kernels(extract=5.0, knn_batch_mfma=4.0), 1_280_000, 1, "nowhere")
    assert e["kernel"] == "extract" and e["bound"] == "alu" and e["peak"] == 157.3
    assert e["achieved"] == pytest.approx(1.28e6 * 100_352 / 5.0e-3 / 1e12)
    assert e["frac_of_dot4_peak"] == pytest.approx(e["achieved"] / bench.PEAK_DOT4_TOPS)
    i8 = bench.roofline_of(kernels(knn_mfma=1.0), 0, 10**8, "nowhere")
    assert i8["peak"] == 5000.0 and i8["achieved"] == pytest.approx(1e8 * 1024 / 1e-3 / 1e12)
    pc = bench.roofline_of(kernels(knn_popcount=1.0), 0, 10**8, "nowhere")
    assert pc["bound"] == "alu" and pc["peak"] == pytest.approx(256 * 64 * 2.4 / 1000)


def test_peaks_are_the_published_and_derived_figures():
    assert bench.PEAK_INT_TOPS == pytest.approx(39.3216)
    assert bench.PEAK_DOT4_TOPS == pytest.approx(8 * 39.3216)
    assert bench.EXTRACT_OPS_PER_DESC == 100_352 and bench.MATCH_OPS_PER_PAIR == 1024


def write_traffic_record(root, source_text, kernel="extract", workload="sfm"):
    src = os.path.join("paper_1609_03986_amd", "csrc", "k.hip")
    os.makedirs(os.path.join(root, os.path.dirname(src)))
    os.makedirs(os.path.join(root, "profiles"))
    with open(os.path.join(root, src), "w") as f:
        f.write(source_text)
    doc = {"kernels": {"%s@%s" % (kernel, workload): {
        "read_bytes_per_launch": 1000.0, "write_bytes_per_launch": 24.0, "source": src,
        "source_sha256": hashlib.sha256(source_text.encode()).hexdigest()}}}
    with open(os.path.join(root, "profiles", "traffic.json"), "w") as f:
        json.dump(doc, f)
    return os.path.join(root, src)


def test_recorded_traffic_is_dropped_once_the_source_changes(tmp_path, monkeypatch):
    src = write_traffic_record(str(tmp_path), "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("extract", "sfm") == 1024.0
    assert bench.recorded_traffic("extract", "hd") is None
    assert bench.recorded_traffic("knn_fp4", "sfm") is None
    with open(src, "a") as f:
        f.write("// a comment\n")
    assert bench.recorded_traffic("extract", "sfm") is None


def test_the_committed_traffic_records_name_existing_sources():
    doc = json.load(open(os.path.join(bench.ROOT, "profiles", "traffic.json")))
    assert doc["calibration"]["copy_bytes"] == 64 << 20
    for key, rec in doc["kernels"].items():
        assert "@" in key
        assert os.path.exists(os.path.join(bench.ROOT, rec["source"])), key
        assert rec["read_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] >= 0


def test_short_kernel_names():
    assert ps.short("void latch::(anonymous namespace)::knn_fp4_kernel<3>(latch::SplitArgs)") == \
        "knn_fp4_kernel<3>"
    assert ps.short("void latch::(anonymous namespace)::extract_kernel<true>(latch::(anonymous "
                    "namespace)::ImageSource, float4 const*)") == "extract_kernel<true>"
    assert ps.launch_of("knn_batch_fp4_kernel<3>") == ("knn_batch_fp4", "knn.hip")
    assert ps.launch_of("order_scan_kernel") == ("extract_order", "order.hip")
    assert ps.launch_of("__amd_rocclr_copyBuffer") == (None, None)


FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
          "End_Timestamp"]


def counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter,
                        "Counter_Value": value, "Start_Timestamp": 1000 * i,
                        "End_Timestamp": 1000 * i + 500})
    return str(path)


def test_traffic_calibrates_by_the_copy_and_groups_kernels_into_launches(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    ext = "void latch::(anonymous namespace)::extract_kernel<true>(int)"
    orders = ["void latch::(anonymous namespace)::order_%s_kernel(int)" % s
              for s in ("count", "scan")]
    fetch = counter_csv(tmp_path / "f.csv", [(copy, "FETCH_SIZE", 32768.0), (copy, "FETCH_SIZE", 8.0),
                                            (ext, "FETCH_SIZE", 100.0), (ext, "FETCH_SIZE", 300.0),
                                            (orders[0], "FETCH_SIZE", 10.0),
                                            (orders[1], "FETCH_SIZE", 6.0)])
    write = counter_csv(tmp_path / "w.csv", [(copy, "WRITE_SIZE", 65536.0), (ext, "WRITE_SIZE", 50.0),
                                            (ext, "WRITE_SIZE", 50.0), (orders[0], "WRITE_SIZE", 1.0),
                                            (orders[1], "WRITE_SIZE", 3.0)])
    out = tmp_path / "traffic.json"

    class Args:
        fetch_copy, write_copy, workload, json = fetch, write, "toy", str(out)
    Args.fetch, Args.write = fetch, write
    text = ps.traffic(Args)
    doc = json.load(open(out))
    # 64 MiB copied: FETCH_SIZE reads half the bytes, WRITE_SIZE all of them.
    assert doc["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert doc["calibration"]["write_factor"] == pytest.approx(1.0)
    e = doc["kernels"]["extract@toy"]
    assert e["read_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2)     # mean of 100 and 300 KiB
    assert e["write_bytes_per_launch"] == pytest.approx(50.0 * 1024)
    src = os.path.join(ps.ROOT, e["source"])
    assert e["source_sha256"] == hashlib.sha256(open(src, "rb").read()).hexdigest()
    o = doc["kernels"]["extract_order@toy"]                # the order's kernels are one launch
    assert o["read_bytes_per_launch"] == pytest.approx(16.0 * 1024 * 2)
    assert o["write_bytes_per_launch"] == pytest.approx(4.0 * 1024)
    assert "| extract |" in text and "Calibration" in text
