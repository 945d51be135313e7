"""The rocprofv3 summariser on synthetic CSV files: HBM traffic scaled by the
calibration kernels (copy x2 for 128-byte requests, sum x1, fill x1), only
the library's kernels kept, launches counted per kernel; kernel statistics
merged by short name; busy and overlapping time of a kernel trace."""
import csv
import os

import pytest

from paper_1404_3448_amd import profsum

GIB = 1 << 30


def write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def counter_dir(tmp_path, name, counter, recs):
    d = tmp_path / name
    write_csv(str(d / "x" / "pmc_counter_collection.csv"), ["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                                            "Counter_Value"],
              [(i, k, counter, kib) for i, (k, kib) in enumerate(recs)])
    return str(d)


def test_short_names():
    assert profsum.short("void lor::(anonymous namespace)::k_radix_scatter<unsigned int, 24, false>(unsigned "
                         "int const*, ...)") == "k_radix_scatter"
    assert profsum.short("lor::k_merge(int)") == "k_merge"
    assert profsum.short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_traffic_scaling_and_filter(tmp_path):
    gib_kib = GIB / 1024
    fetch = counter_dir(tmp_path, "f", "FETCH_SIZE", [
        ("__amd_rocclr_copyBuffer", gib_kib / 2),            # 128-byte requests: half the bytes counted
        ("at::native::reduce_kernel<...>", gib_kib),         # 64-byte requests
        ("lor::(anonymous namespace)::k_radix_scatter<unsigned int, 24, false>(...)", 1000.0),
        ("lor::(anonymous namespace)::k_radix_scatter<unsigned long, 16, true>(...)", 3000.0),
        ("lor::(anonymous namespace)::k_merge<unsigned char, 4>(...)", 500.0),
        ("some_other_kernel", 99999.0),
    ])
    write = counter_dir(tmp_path, "w", "WRITE_SIZE", [
        ("__amd_rocclr_copyBuffer", gib_kib),
        ("at::native::vectorized_elementwise_kernel<FillFunctor>", gib_kib),
        ("lor::(anonymous namespace)::k_radix_scatter<unsigned int, 24, false>(...)", 700.0),
        ("lor::(anonymous namespace)::k_radix_scatter<unsigned long, 16, true>(...)", 900.0),
        ("lor::(anonymous namespace)::k_merge<unsigned char, 4>(...)", 100.0),
    ])
    doc = profsum.traffic(fetch, write, "abc")
    cal = doc["calibration"]
    assert cal["fetch_factor"] == pytest.approx(2.0)
    assert cal["fetch_factor_lo"] == pytest.approx(1.0)
    assert cal["write_factor"] == pytest.approx(1.0)
    assert doc["source_sha256"] == "abc"
    k = doc["kernels"]
    assert set(k) == {"k_radix_scatter", "k_merge"}          # only the library's kernels, by short name
    rs = k["k_radix_scatter"]
    assert rs["launches"] == 2
    assert rs["read_bytes"] == pytest.approx(2 * 4000.0 * 1024)
    assert rs["read_bytes_lo"] == pytest.approx(4000.0 * 1024)
    assert rs["write_bytes"] == pytest.approx(1600.0 * 1024)
    assert k["k_merge"]["launches"] == 1
    assert list(k)[0] == "k_radix_scatter"                    # ordered by bytes, largest first
    table = profsum.traffic_table(doc)
    assert "| k_radix_scatter | 2 |" in table


def test_traffic_needs_calibration_kernels(tmp_path):
    fetch = counter_dir(tmp_path, "f", "FETCH_SIZE", [("lor::k_merge(int)", 1.0)])
    write = counter_dir(tmp_path, "w", "WRITE_SIZE", [("lor::k_merge(int)", 1.0)])
    with pytest.raises(SystemExit):
        profsum.traffic(fetch, write, "abc")


def test_stats_merges_by_short_name(tmp_path):
    p = str(tmp_path / "s.csv")
    write_csv(p, ["Name", "Calls", "TotalDurationNs"], [
        ("lor::k_radix_scatter<unsigned int, 24, false>(...)", 3, 3_000_000),
        ("lor::k_radix_scatter<unsigned long, 16, true>(...)", 1, 1_000_000),
        ("lor::k_merge<unsigned char, 4>(...)", 2, 6_000_000),
    ])
    out = profsum.stats(p).splitlines()
    assert out[2] == "| k_merge | 2 | 6.00 | 3.0000 | 60.0 |"
    assert out[3] == "| k_radix_scatter | 4 | 4.00 | 1.0000 | 40.0 |"
    assert out[-1] == "All kernels: 10.0 ms."


def test_trace_busy_overlap_and_phases(tmp_path):
    p = str(tmp_path / "t.csv")
    ms = 1_000_000
    # [0,4) and [2,6) overlap for 2 ms on two streams; [20,21) after an idle gap
    write_csv(p, ["Start_Timestamp", "End_Timestamp", "Stream_Id"],
              [(0, 4 * ms, 1), (2 * ms, 6 * ms, 2), (20 * ms, 21 * ms, 1)])
    one = profsum.trace(p)
    assert "3 kernels from 2 streams over 21.0 ms" in one
    assert "GPU busy (some kernel running) 7.0 ms" in one and "idle 14.0 ms" in one
    assert "two or more kernels at once 2.0 ms" in one
    phases = profsum.trace(p, split_gap_ms=5.0).splitlines()
    assert len(phases) == 2
    assert phases[0].startswith("phase 0: 2 kernels from 2 streams over 6.0 ms")
    assert phases[1].startswith("phase 1: 1 kernels from 1 streams over 1.0 ms")
