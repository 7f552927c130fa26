"""Host checks of the benchmark's roofline arithmetic (no GPU): achieved
bandwidth is the algorithmic bytes of the dominant kernel per launch divided by
its mean launch time, and the recorded traffic is used only for the kernel
source it was measured on."""
import json

import pytest

import bench


def _peel_stats():
    return {"kernel_ms": {"support_init": 1.0, "jump_min": 2.0, "mark": 3.0,
                          "level_events": 40.0, "support_update": 10.0, "advance": 2.0},
            "kernel_launches": {"support_init": 1, "jump_min": 100, "mark": 100,
                                "level_events": 100, "support_update": 100, "advance": 100},
            "work": {"level_items": 1000, "level_slots": 2000, "level_candidates": 3000,
                     "level_probes": 4000, "level_drops": 5000, "support_items": 6,
                     "support_slots": 7, "support_hits": 8}}


def test_peel_roofline_arithmetic():
    r = bench.roofline_from_stats(_peel_stats(), "no_such_workload")
    alg = 1000 * 16 + 2000 * 8 + 3000 * 32 + 4000 * 16 + 5000 * 48
    assert r["kernel"] == "k_level" and r["launches"] == 100
    assert r["alg_bytes_per_launch"] == pytest.approx(alg / 100)
    assert r["achieved"] == pytest.approx(alg / 100 / (0.4e-3) / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["traffic"] is None


def test_support_roofline_arithmetic():
    st = _peel_stats()
    st["kernel_ms"]["support_update"] = 80.0
    r = bench.roofline_from_stats(st, "no_such_workload")
    alg = 6 * 16 + 7 * 20 + 8 * 8
    assert r["kernel"] == "k_support"
    assert r["alg_bytes_per_launch"] == pytest.approx(alg / 100)


def test_hindex_roofline_arithmetic():
    st = {"rounds": 4,
          "kernel_ms": {"a": 1.0, "b": 2.0, "c": 8.0, "d": 0.5},
          "kernel_launches": {"a": 1, "b": 4, "c": 4, "d": 4},
          "work": {"k0": 10, "k1": 20, "k2": 30, "k3": 40, "k4": 50, "k5": 60, "k6": 7000,
                   "k7": 80}}
    m = 100
    r = bench._hx_roofline(st, m)
    alg = 7000 + 80 * 8 + 4 * m * 28
    assert r["kernel"] == "k_hx_edges" and r["launches"] == 4
    assert r["alg_bytes_per_launch"] == pytest.approx(alg / 4)
    assert r["achieved"] == pytest.approx(alg / 4 / 2e-3 / 1e9)


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", tmp_path)
    rec = {"source_sha": bench.kernel_source_sha("k_level"), "bytes_per_launch": 123.0}
    (tmp_path / "traffic_k_level_w.txt").write_text(json.dumps(rec))
    assert bench.recorded_traffic("k_level", "w") == 123.0
    rec["source_sha"] = "0" * 16
    (tmp_path / "traffic_k_level_w.txt").write_text(json.dumps(rec))
    assert bench.recorded_traffic("k_level", "w") is None
    assert bench.recorded_traffic("k_support", "w") is None


def test_whole_run_fields(tmp_path, monkeypatch):
    """Counter fraction = recorded bytes / device time / 8 TB/s; traffic
    efficiency = recorded bytes / B_alg; the recorded bytes count only while
    taken on the current kernel source."""
    monkeypatch.setattr(bench, "PROFILES", tmp_path)
    rec = {"source_sha": bench.kernel_source_sha("k_level"), "bytes_per_decomposition": 4.0e12}
    (tmp_path / "traffic_whole_w.txt").write_text(json.dumps(rec))
    st = {"evaluations": 2.0e9, "alg_bytes": 8.0e14}
    r = bench.whole_run(st, "w", 1000.0)
    assert r["counter_bytes"] == 4.0e12
    assert r["counter_frac"] == pytest.approx(4.0e12 / 1.0 / 8.0e12)
    assert r["traffic_efficiency"] == pytest.approx(4.0e12 / 8.0e14)
    assert r["evaluations_per_s"] == pytest.approx(2.0e9)
    rec["source_sha"] = "0" * 16
    (tmp_path / "traffic_whole_w.txt").write_text(json.dumps(rec))
    r = bench.whole_run(st, "w", 1000.0)
    assert r["counter_bytes"] is None
    assert "counter_frac" not in r and "traffic_efficiency" not in r
    assert r["evaluations_per_s"] == pytest.approx(2.0e9)
