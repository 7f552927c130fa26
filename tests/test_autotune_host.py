"""Host logic of the autotuner: shape buckets, the coordinate search and the
JSON cache (no GPU: the timing function is a stand-in cost surface)."""
import json

from paper_2411_06405_amd import autotune as A


def test_shape_key_buckets():
    k1 = A.shape_key("MI355X", 100_000, 500_000, 2, 6000)
    k2 = A.shape_key("MI355X", 120_000, 600_000, 2, 6500)   # same buckets
    k3 = A.shape_key("MI355X", 100_000, 500_000, 3, 6000)   # other h
    k4 = A.shape_key("MI355X", 400_000, 500_000, 2, 6000)   # other n, avg degree
    assert k1 == k2 and k1 != k3 and k1 != k4
    assert k1.startswith("MI355X|")


def test_search_finds_the_minimum_of_a_separable_surface():
    cost = {("dense_threshold", 4): 3.0, ("dense_threshold", 32): 1.0,
            ("dense_threshold", 256): 2.0, ("dense_threshold", 1 << 30): 5.0}
    calls = []

    def time_fn(t):
        calls.append(dict(t))
        c = cost[("dense_threshold", t["dense_threshold"])] if t["dense_threshold"] else 9.0
        c += {64: 0.5, 128: 0.1}[t["word_bits"]] * {0: 1, 1: 3, 4: 1, 16: 2}[t["edges_per_wave"]]
        return c
    best = A.search(time_fn, repeats=2)
    assert best == {"dense_threshold": 32, "word_bits": 128, "edges_per_wave": 4}
    # 4 dense candidates + 6 (width, edges/wave) pairs, each timed twice
    assert len(calls) == 2 * (len(A.DENSE_THRESHOLDS) + len(A.WIDTHS) * len(A.EDGES_PER_WAVE))


def test_choose_prefers_first_on_ties():
    assert A.choose({"a": 1.0, "b": 1.0, "c": 2.0}) == "a"


def test_cache_round_trip(tmp_path):
    p = tmp_path / "tune.json"
    c = A.Cache(p)
    assert c.get("k") is None
    c.put("k", {"word_bits": 128, "edges_per_wave": 4, "dense_threshold": 32})
    assert json.loads(p.read_text())["k"]["word_bits"] == 128
    assert A.Cache(p).get("k") == {"word_bits": 128, "edges_per_wave": 4, "dense_threshold": 32}
    p.write_text("not json")
    assert A.Cache(p).get("k") is None  # a corrupt cache is ignored


def test_round_search_keeps_the_base_and_picks_the_fastest_grid():
    base = {"dense_threshold": 32, "word_bits": 64, "edges_per_wave": 0}
    seen = []

    def time_fn(t):
        seen.append(t["grid_blocks"])
        assert {k: t[k] for k in base} == base
        return {4 * 256: 3.0, 8 * 256: 1.0, 16 * 256: 2.0}[t["grid_blocks"]]
    best = A.search_rounds(time_fn, base, num_cu=256, repeats=2)
    assert best == dict(base, grid_blocks=8 * 256)
    assert sorted(set(seen)) == [p * 256 for p in A.GRID_PER_CU] and len(seen) == 6
