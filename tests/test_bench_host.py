"""Host logic of bench.py that needs no GPU: the per-iteration block schedule
it times beside constant nb, and the gate that keeps a traffic figure off the
bench line when the GEMM source differs from the one the counters measured
(or the summary is missing)."""
import bench


def test_lead_schedule_covers_three_eighths_of_the_order_in_double_blocks():
    assert bench.lead_schedule(16384, 256) == [512] * 12
    assert bench.lead_schedule(4096, 256) == [512] * 3
    for n, nb in [(16384, 128), (8192, 256), (10000, 192), (300, 64)]:
        s = bench.lead_schedule(n, nb)
        assert all(b == 2 * nb for b in s)
        assert sum(s) <= max(3 * n // 8, 2 * nb)
        assert sum(s) + 2 * nb > 3 * n // 8 or len(s) == 1
    assert bench.lead_schedule(256, 256) == [512]   # one block, trimmed to the order by the library


def test_traffic_record_is_tied_to_the_gemm_source(tmp_path, monkeypatch):
    import hashlib
    import json
    import re

    text = open(bench.TRAFFIC_FILE).read()
    rec = json.loads(re.search(r"TRAFFIC_JSON:\s*(\{.*\})", text).group(1))
    src = tmp_path / "gemm.hip"
    src.write_bytes(b"// a kernel source the counters were not taken on\n")
    monkeypatch.setattr(bench, "GEMM_SRC", str(src))
    assert bench.traffic_record() is None
    # the same summary against a source whose hash it records: returned as is
    fake = tmp_path / "traffic.md"
    rec["source_sha1"] = hashlib.sha1(src.read_bytes()).hexdigest()
    fake.write_text("counters\nTRAFFIC_JSON: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(fake))
    got = bench.traffic_record()
    assert got == rec and got["fetch_bytes_per_step"] > 0 and got["write_bytes_per_step"] > 0
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.traffic_record() is None


def test_mfma_record_is_tied_to_the_gemm_source(tmp_path, monkeypatch):
    rec = bench.mfma_record()
    assert rec is not None
    frac = rec["kernels"]["k_gemm_queue_whole"]["mfma_busy_frac"]
    assert 0.0 < frac <= 1.0
    src = tmp_path / "gemm.hip"
    src.write_bytes(b"// another kernel source\n")
    monkeypatch.setattr(bench, "GEMM_SRC", str(src))
    assert bench.mfma_record() is None


def test_grid_summary_on_synthetic_counter_runs(tmp_path):
    """rocprof_summary grid: the time-weighted matrix-core busy fraction
    (busy cycles over active cycles summed over dispatches, over the same ratio
    of the calibration kernel), the calibrated bytes (each counter scaled by
    what it reads for the known copy in its own run) and the rate over the
    summed durations, on hand-made CSV files with a known answer."""
    import csv

    from paper_1611_06365_amd import rocprof_summary as R

    copy = "at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<double, double, double, " \
           "at::native::MulFunctor"

    def counters(d, rows):
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writerows(rows)

    cal, a, b, c = (tmp_path / x for x in ("cal", "a", "b", "c"))
    counters(cal, [(1, "k_mfma_peak", "SQ_VALU_MFMA_BUSY_CYCLES", 1000), (1, "k_mfma_peak", "GRBM_GUI_ACTIVE", 10)])
    # two dispatches of the kernel: one busy for half its active cycles, one (a helper that found no
    # work) with no busy cycles; time-weighted: 500 / (10 + 10) / 100 = 0.25
    counters(a, [(5, "mlu::k_x", "SQ_VALU_MFMA_BUSY_CYCLES", 500), (5, "mlu::k_x", "GRBM_GUI_ACTIVE", 10),
                 (5, "mlu::k_x", "SQ_INSTS_VALU_MFMA_MOPS_F64", 2000000), (6, "mlu::k_x", "SQ_VALU_MFMA_BUSY_CYCLES", 0),
                 (6, "mlu::k_x", "GRBM_GUI_ACTIVE", 10), (6, "mlu::k_x", "SQ_INSTS_VALU_MFMA_MOPS_F64", 0)])
    with open(a / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writerows([(5, "mlu::k_x", 0, 3000), (6, "mlu::k_x", 5000, 6000)])
    counters(b, [(5, "mlu::k_x", "FETCH_SIZE", 1000), (6, "mlu::k_x", "FETCH_SIZE", 0), (9, copy, "FETCH_SIZE", 512)])
    counters(c, [(5, "mlu::k_x", "WRITE_SIZE", 300), (6, "mlu::k_x", "WRITE_SIZE", 100), (9, copy, "WRITE_SIZE", 1024)])
    rows = R.grid(str(cal), [("cfg", str(a), str(b), str(c))], ["k_x"], copy_bytes=1 << 20,
                  copy_kernel=r"AUnaryFunctor<double, double, double, .*MulFunctor")
    assert len(rows) == 1
    r = rows[0]
    assert r["dispatches"] == 2 and r["avg_us"] == 2.0
    assert r["mfma_busy_frac"] == 0.25
    assert r["f64_gflop"] == 0.512   # 512 flops per MOPS, 1e6 MOPS per dispatch on average
    # FETCH: copy reads 512 KiB of 1 MiB -> scale 2; mean 500 KiB -> 1 024 000 bytes
    assert r["fetch_bytes"] == 1024000
    # WRITE: copy reads 1024 KiB of 1 MiB -> scale 1; mean 200 KiB -> 204 800 bytes
    assert r["write_bytes"] == 204800
    assert r["hbm_gbs"] == round((1024000 + 204800) / 2000.0, 1)
