"""The rocprofv3 summary helpers (CPU only): kernel-trace table, HBM traffic
from FETCH_SIZE / WRITE_SIZE scaled by a calibration copy, and the stored
measurement's match to the kernel source."""
import csv
import json

from paper_2303_04353_amd import profiling as pf


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_trace_table_names_and_units(tmp_path):
    p = tmp_path / "stats.csv"
    _write(p, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
           [["void ddk::cascade_kernel<false, false>(double const*, double const*)", 7, 7e9, 1.654e8, 60.0,
             1.650e8, 1.660e8],
            ["(anonymous namespace)::helper(int)", 2, 10, 5.0, 0.1, 4.0, 6.0]])
    t = pf.trace_table(str(p)).splitlines()
    assert t[2].startswith("| ddk::cascade_kernel<false, false> | 7 | 165400.0 |")
    assert t[3].startswith("| helper | 2 | 0.0 |")


# the headline product kernel as rocprofv3 names it (buffer-load staging form)
PROD = "void ddk::cascade_kernel<false, false, ddk::(anonymous namespace)::Shape<64, 64, 7>, true>"


def test_traffic_scales_by_the_calibration_copy(tmp_path):
    mib = 1024
    copy_bytes = mib << 20
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy reads each byte once but FETCH_SIZE counts half of it (x2),
    # WRITE_SIZE counts it all (x1); the product kernel fetches 10 GiB, writes 1 GiB
    fetch = [["vectorized_elementwise_kernel<copy>", "FETCH_SIZE", copy_bytes / 2 / 1024],
             [PROD + "(double const*)", "FETCH_SIZE", 5 * (1 << 30) / 1024],
             [PROD + "(double const*)", "FETCH_SIZE", 5 * (1 << 30) / 1024],
             ["void ddk::cascade_kernel<false, true, ddk::(anonymous namespace)::Shape<64, 64, 7>, true>(double const*)",
              "FETCH_SIZE", 1.0],
             ["void ddk::cascade_kernel<false, false, ddk::(anonymous namespace)::Shape<32, 64, 7>, true>(double const*)",
              "FETCH_SIZE", 1.0]]
    write = [["vectorized_elementwise_kernel<copy>", "WRITE_SIZE", copy_bytes / 1024],
             [PROD + "(double const*)", "WRITE_SIZE", (1 << 30) / 1024]]
    _write(tmp_path / "f.csv", hdr, fetch)
    _write(tmp_path / "w.csv", hdr, write)
    r = pf.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), mib, 8, 8, 8)
    assert abs(r["fetch_scale"] - 2.0) < 1e-12 and abs(r["write_scale"] - 1.0) < 1e-12
    assert abs(r["fetch_bytes_per_launch"] - 10 * (1 << 30)) < 1
    assert abs(r["bytes_per_launch"] - 11 * (1 << 30)) < 1
    assert r["dispatches"] == [2, 1] and r["source_sha256_16"] == pf.source_hash()
    assert r["kernel"] == "cascade_kernel<false, false, Shape<64, 64, 7>, true>"
    # a stored measurement counts only for the same shape and kernel source
    out = tmp_path / "t.json"
    out.write_text(json.dumps(r))
    assert pf.load_traffic(str(out), 8, 8, 8) == r["bytes_per_launch"]
    assert pf.load_traffic(str(out), 8, 8, 16) is None
    r["source_sha256_16"] = "0" * 16
    out.write_text(json.dumps(r))
    assert pf.load_traffic(str(out), 8, 8, 8) is None


def test_counter_summary_clock_and_busy_shares(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
           "End_Timestamp"]
    # a 1 ms dispatch: 1.5e6 cycles on each of 8 XCDs = 1.5 GHz; the matrix cores of
    # the 1024 SIMDs busy for 0.75 of those cycles
    busy = 0.75 * 1024 * 1.5e6
    sq = [[1, "void k<1>(int)", "GRBM_GUI_ACTIVE", 8 * 1.5e6, 0, 1000000],
          [1, "void k<1>(int)", "SQ_VALU_MFMA_BUSY_CYCLES", busy, 0, 1000000],
          [1, "void k<1>(int)", "SQ_WAVE_CYCLES", 1000, 0, 1000000],
          [1, "void k<1>(int)", "SQ_WAIT_ANY", 250, 0, 1000000],
          # a second dispatch, 3 ms at 2.4 GHz, matrix cores idle
          [2, "void k<1>(int)", "GRBM_GUI_ACTIVE", 8 * 7.2e6, 0, 3000000],
          [2, "void k<1>(int)", "SQ_VALU_MFMA_BUSY_CYCLES", 0, 0, 3000000]]
    cache = [[1, "void k<1>(int)", "TCC_HIT_sum", 3, 0, 10], [1, "void k<1>(int)", "TCC_MISS_sum", 1, 0, 10],
             [2, "vectorized_elementwise_kernel<copy>", "TCC_HIT_sum", 0, 0, 10]]
    fetch = [[1, "vectorized_elementwise_kernel<copy>", "FETCH_SIZE", (1 << 30) / 2 / 1024, 0, 10],
             [2, "void k<1>(int)", "FETCH_SIZE", 1024.0, 0, 10]]
    for name, rows in (("sq", sq), ("cache", cache), ("fetch", fetch)):
        _write(tmp_path / (name + ".csv"), hdr, rows)
    s = pf.counter_summary([str(tmp_path / n) for n in ("sq.csv", "cache.csv", "fetch.csv")], copy_mib=1024)
    r = s["k<1>"]
    # (1.5e6 + 7.2e6) cycles over 4 ms
    assert abs(r["clock_ghz"] - 8.7e6 / 4e-3 / 1e9) < 1e-12
    assert abs(r["mfma_busy_of_active"] - busy / (1024 * 8.7e6)) < 1e-12
    assert abs(r["mfma_busy_of_peak_clock"] - busy / (1024 * 2.4e9 * 4e-3)) < 1e-12
    assert r["sq_wait_any_per_wave_cycle"] == 0.25 and r["l2_hit_rate"] == 0.75
    # FETCH_SIZE of the copy reads half its bytes: the factor is 2
    assert abs(r["fetch_bytes"] - 2 * 1024 * 1024) < 1e-6
    assert r["dispatches"] == 4
    t = pf.counter_table(s, "k<1>").splitlines()
    assert len(t) == 3 and t[2].startswith("| k<1> | 4 | 2.17 | 0.129 | 0.117 | 0.250 | - | 0.750 | 0.00 |")
