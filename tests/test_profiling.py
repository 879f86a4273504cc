"""Host logic of the rocprofv3 summaries: copy calibration of the traffic
counters, the kernel-name filter, staleness of a record, and the table of the
integer passes (synthetic counter files, no GPU)."""
import csv
import os

from paper_2605_10135_amd import profiling

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, value, dur) in enumerate(rows):
            r = {k: 0 for k in FIELDS}
            r.update(Dispatch_Id=i + 1, Kernel_Name=name, Counter_Name=counter, Counter_Value=value,
                     Start_Timestamp=1000, End_Timestamp=1000 + dur)
            w.writerow(r)


def test_traffic_record_is_copy_calibrated_filtered_and_hashed(tmp_path):
    calib_kib = profiling.CALIB_BYTES / 1024.0
    # the counters read half the copy's bytes on fetch and all of them on write
    _write(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", calib_kib / 2, 10),
                                             ("void sg::batch::dist_topk_batched_kernel<1>(x)", 1000.0, 10),
                                             ("void sg::knn::dist_topk_kernel<1>(x)", 9999.0, 10)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", calib_kib, 10),
                                              ("void sg::batch::dist_topk_batched_kernel<1>(x)", 10.0, 10),
                                              ("void sg::knn::dist_topk_kernel<1>(x)", 7777.0, 10)])
    out = tmp_path / "rec.txt"
    profiling.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), "f", "w", "dist_topk_batched")
    rec = profiling.read_traffic(str(out))
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["fetch_bytes"] == 1000.0 * 1024 * 2 and rec["write_bytes"] == 10.0 * 1024
    assert rec["bytes"] == rec["fetch_bytes"] + rec["write_bytes"]
    # a record taken on other kernel sources is stale
    text = out.read_text().replace(profiling.kernel_sha(), "0" * 64)
    out.write_text(text)
    assert profiling.read_traffic(str(out)) is None
    assert profiling.read_traffic(str(tmp_path / "missing.txt")) is None


def test_integer_table_lists_each_filtered_kernel(tmp_path):
    calib_kib = profiling.CALIB_BYTES / 1024.0
    _write(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", calib_kib, 5),
                                             ("void sg::prune::detour_kernel<1, 256>(a)", 2048.0, 3_000_000),
                                             ("void sg::prune::detour_kernel<1, 256>(a)", 4096.0, 1_000_000),
                                             ("sg::merge::merge_kernel(b)", 1024.0, 500_000)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", calib_kib, 5),
                                              ("void sg::prune::detour_kernel<1, 256>(a)", 1024.0, 3_000_000),
                                              ("void sg::prune::detour_kernel<1, 256>(a)", 1024.0, 1_000_000),
                                              ("sg::merge::merge_kernel(b)", 0.0, 500_000)])
    out = tmp_path / "t.md"
    profiling.integer_table(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), "f", "w",
                            "prune::detour,merge::merge_kernel")
    rows = [l for l in out.read_text().splitlines() if l.startswith("| `")]
    assert len(rows) == 2
    det = [c.strip() for c in rows[0].split("|")[1:-1]]
    # mean of 2 MiB and 4 MiB fetched, 1 MiB written, 2 ms per dispatch
    assert det[1] == "2" and det[2] == "%.1f" % (3072 * 1024 / 1e6) and det[3] == "%.1f" % (1024 * 1024 / 1e6)
    assert det[4] == "2.000"
    assert os.path.exists(out)


def test_bench_takes_the_record_of_the_shape_it_chose(tmp_path, monkeypatch):
    # one record per pinned launch shape; the bench line takes the one whose
    # variant is the shape its autotuner chose, and none for an unrecorded shape
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    calib_kib = profiling.CALIB_BYTES / 1024.0
    (tmp_path / "profiles").mkdir()
    for v, kib in ((2, 1000.0), (3, 3000.0)):
        _write(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", calib_kib, 10),
                                                 ("void sg::batch::dist_topk_batched_kernel<%d>(x)" % v, kib, 10)])
        _write(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", calib_kib, 10),
                                                  ("void sg::batch::dist_topk_batched_kernel<%d>(x)" % v, 0.0, 10)])
        profiling.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                          str(tmp_path / "profiles" / ("dist_topk_wl_v%d_traffic.txt" % v)), "f", "w",
                          "dist_topk_batched", str(v))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    r2, r3 = bench.traffic_of("wl", 2), bench.traffic_of("wl", 3)
    assert r2["variant"] == 2 and r2["fetch_bytes"] == 1000.0 * 1024 and "<2>" in r2["kernels"]
    assert r3["variant"] == 3 and r3["fetch_bytes"] == 3000.0 * 1024 and "<3>" in r3["kernels"]
    assert bench.traffic_of("wl", 0) is None
