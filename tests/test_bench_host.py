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
