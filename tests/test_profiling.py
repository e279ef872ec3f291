"""Host logic of the profile summaries: counters summed over their
instances within a dispatch, HBM bytes scaled by what the same counter reads
for a copy of known size, counter means and ratios per kernel."""
import csv

import pytest

from paper_2006_13631_amd import profiling as P

FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, k, c, v in rows:
            w.writerow({"Correlation_Id": d, "Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c,
                        "Counter_Value": v})
    return str(path)


KERNEL = "void ns::k_stream_collide2<double, double>(ns::CaseView<double, double>, int)"
LONGER = "void ns::k_stream_collide2_probe<double>(double*)"


def test_per_dispatch_sums_instances(tmp_path):
    p = _csv(tmp_path / "a.csv", [(1, KERNEL, "FETCH_SIZE", 10.0), (1, KERNEL, "FETCH_SIZE", 5.0),
                                  (2, KERNEL, "FETCH_SIZE", 7.0), (2, KERNEL, "WRITE_SIZE", 99.0)])
    per = P._per_dispatch(p, "FETCH_SIZE")
    assert sorted(per[KERNEL]) == [7.0, 15.0]


def test_traffic_scaled_by_the_copy(tmp_path):
    copy = P.COPY_KERNEL
    # the copy of 1 MiB reads as 512 KiB fetched and 1024 KiB written
    f = _csv(tmp_path / "f.csv", [(1, copy, "FETCH_SIZE", 512.0), (2, KERNEL, "FETCH_SIZE", 100.0),
                                  (3, KERNEL, "FETCH_SIZE", 300.0), (4, LONGER, "FETCH_SIZE", 1e6)])
    w = _csv(tmp_path / "w.csv", [(1, copy, "WRITE_SIZE", 1024.0), (2, KERNEL, "WRITE_SIZE", 50.0),
                                  (3, KERNEL, "WRITE_SIZE", 50.0)])
    r = P.traffic(f, w, "k_stream_collide2", 1 << 20)
    assert r["FETCH_SIZE"]["copy_scale"] == pytest.approx(2.0)
    assert r["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0)  # mean 200 KiB, x2
    assert r["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(50.0 * 1024)
    assert r["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0 + 50.0 * 1024)
    assert r["FETCH_SIZE"]["dispatches"] == 2  # the longer name is another kernel


def test_traffic_skips_leading_dispatches(tmp_path):
    copy = P.COPY_KERNEL
    # dispatch ids out of order in the file: the skip follows dispatch order
    f = _csv(tmp_path / "f.csv", [(3, KERNEL, "FETCH_SIZE", 100.0), (1, copy, "FETCH_SIZE", 512.0),
                                  (2, KERNEL, "FETCH_SIZE", 900.0), (4, KERNEL, "FETCH_SIZE", 300.0)])
    w = _csv(tmp_path / "w.csv", [(1, copy, "WRITE_SIZE", 1024.0), (2, KERNEL, "WRITE_SIZE", 70.0),
                                  (3, KERNEL, "WRITE_SIZE", 50.0), (4, KERNEL, "WRITE_SIZE", 50.0)])
    r = P.traffic(f, w, "k_stream_collide2", 1 << 20, skip=1)
    assert r["FETCH_SIZE"]["dispatches"] == 2 and r["FETCH_SIZE"]["skipped"] == 1
    assert r["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0)
    assert r["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(50.0 * 1024)


def test_traffic_needs_both_kernels(tmp_path):
    f = _csv(tmp_path / "f.csv", [(2, KERNEL, "FETCH_SIZE", 100.0)])
    with pytest.raises(SystemExit):
        P.traffic(f, f, "k_stream_collide2", 1 << 20)


def test_counter_means_and_ratios(tmp_path):
    rows = []
    for d, (waves, cyc, wait, lds, conf) in enumerate([(10, 1000, 600, 40, 80), (10, 3000, 1800, 40, 80)]):
        for c, v in (("SQ_WAVES", waves), ("SQ_WAVE_CYCLES", cyc), ("SQ_WAIT_INST_ANY", wait),
                     ("SQ_INSTS_LDS", lds), ("SQ_LDS_BANK_CONFLICT", conf)):
            rows.append((d + 1, KERNEL, c, v))
    text = P.counters(_csv(tmp_path / "c.csv", rows), ["k_stream_collide2<double", "k_absent"])
    assert "(2 dispatches)" in text
    assert "SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES = 0.600" in text
    assert "SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS = 2.000" in text
    assert "k_absent: no dispatch" in text
