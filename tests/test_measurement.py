"""The measurement helpers on the CPU: the reduction of rocprofv3 counter
files to HBM bytes per launch (calibrated by the 1 GiB copies in the same
run) and the rule that a stored figure is reported only while the kernel
sources it was taken on are unchanged."""
import csv
import json

import pytest

from paper_2502_08382_amd import traffic

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value,
                        "Start_Timestamp": 1000 * i, "End_Timestamp": 1000 * i + 500})


def _files(tmp_path):
    gib_kib = (1 << 30) / 1024
    # FETCH_SIZE reads half of a copy's bytes, WRITE_SIZE all of them; small
    # copies (set-up) and other kernels must not enter the calibration
    fetch = [("copyBuffer", gib_kib / 2)] * 3 + [("copyBuffer", 3.0), ("other_kernel", 77.0),
                                                 ("apply_seg_kernel<double, 4, 4, true>", 1000.0),
                                                 ("apply_seg_kernel<double, 4, 4, true>", 1002.0)]
    write = [("copyBuffer", gib_kib)] * 3 + [("apply_seg_kernel<double, 4, 4, true>", 10.0),
                                            ("apply_seg_kernel<double, 4, 4, true>", 12.0)]
    fp, wp = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    return fp, wp


def test_summarize_scales_by_the_copy_calibration(tmp_path):
    fp, wp = _files(tmp_path)
    rec = traffic.summarize(str(fp), str(wp), kernel="apply_seg_kernel")
    assert rec["dispatches"] == 2
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["fetch_bytes"] == pytest.approx(1001.0 * 1024 * 2.0)
    assert rec["write_bytes"] == pytest.approx(11.0 * 1024)
    assert rec["traffic_bytes"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["fetch_kib"] == [1000.0, 1002.0] and rec["source_sha256_16"] == traffic.kernel_source_hash()


def test_summarize_needs_the_copies_and_the_kernel(tmp_path):
    fp, wp = _files(tmp_path)
    with pytest.raises(ValueError):
        traffic.summarize(str(fp), str(wp), kernel="no_such_kernel")
    _write(fp, "FETCH_SIZE", [("apply_seg_kernel", 5.0)])
    with pytest.raises(ValueError):
        traffic.summarize(str(fp), str(wp), kernel="apply_seg_kernel")


def test_lookup_reports_only_records_of_the_current_sources(tmp_path, monkeypatch):
    store = tmp_path / "traffic.json"
    cur = traffic.kernel_source_hash()
    store.write_text(json.dumps({"now": {"traffic_bytes": 1.0, "source_sha256_16": cur},
                                 "stale": {"traffic_bytes": 2.0, "source_sha256_16": "0" * 16}}))
    monkeypatch.setattr(traffic, "STORE", str(store))
    assert traffic.lookup("now")["traffic_bytes"] == 1.0
    assert traffic.lookup("stale") is None and traffic.lookup("missing") is None

