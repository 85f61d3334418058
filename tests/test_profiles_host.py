"""The committed counter summaries are well formed (CPU).

profiles/pmc_traffic.json carries, per profiled workload and pass, the bytes
per launch that left the L2 (rocprofv3 FETCH_SIZE and WRITE_SIZE, divided by
the factors a 1 GiB copy gives them), the algorithmic bytes of the pass, and
the kernel-source hash and the geometry they were taken on; bench.py
attaches them to its per-pass figures only while that hash matches the
sources and the geometry matches the one in effect.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_traffic_file_structure():
    d = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))
    assert len(d["kernel_source_hash"]) == 16
    cal = d["calibration"]
    assert 0.4 < cal["FETCH_SIZE"] < 1.1 and 0.9 < cal["WRITE_SIZE"] < 1.1
    assert set(d["workloads"]) == {"plain", "batched", "large"}
    for name, w in d["workloads"].items():
        assert os.path.exists(os.path.join(ROOT, w["summary"])), name
        assert len(w["geometry"]) == 4 and w["geometry"][1] in (16, 32, 64), name
        assert set(w["kernels"]) == {"colfwd", "rowconv", "colinv"}
        for k, v in w["kernels"].items():
            # every pass moves at least its algorithmic bytes, and re-reads
            # stay small (twiddle tables, partial lines of the bit arrays)
            ratio = v["hbm_bytes_per_launch"] / v["alg_bytes_per_launch"]
            assert 0.97 < ratio < 1.25, (name, k, ratio)
            assert 0.0 < v["valu_busy"] <= 1.0 and 0.0 < v["fp64_frac"] < 1.0


def test_bench_reads_traffic_only_for_matching_sources(monkeypatch):
    import bench
    d = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: d["kernel_source_hash"])
    want = d["workloads"]["batched"]["kernels"]["rowconv"]["hbm_bytes_per_launch"]
    assert bench.load_traffic("rowconv", "batched") == want
    geom = d["workloads"]["batched"]["geometry"]
    assert bench.load_traffic("rowconv", "batched", geom) == want
    other = [geom[0], 64 if geom[1] != 64 else 32, geom[2], geom[3]]
    assert bench.load_traffic("rowconv", "batched", other) is None
    assert bench.load_traffic("nosuch", "batched") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("rowconv", "batched") is None
