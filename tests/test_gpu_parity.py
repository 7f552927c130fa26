"""GPU parity: the HIP path (through the C ABI) against the plain CPU oracle,
bit-exact on trussness and on the bulk round schedule."""
import numpy as np
import pytest

import oracle
from graphgen import disjoint_union, from_edge_list, gen, workloads as W
from tests.gpu_helpers import assert_exact, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("seed", W.D1_SEEDS)
@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_d1_exact(seed, h):
    assert_exact(W.d1(seed), h)


@pytest.mark.parametrize("tune", [None, {"dense_threshold": 1}, {"dense_threshold": 1 << 30},
                                  {"word_bits": 128, "edges_per_wave": 16},
                                  {"word_bits": 128, "edges_per_wave": 1}])
@pytest.mark.parametrize("h", [1, 2, 3])
def test_support_exact(h, tune):
    # every initial-pass setting (bottom-up / top-down level-2 build, load
    # width, edges per wavefront) gives the oracle's h-support
    import paper_2411_06405_amd as ht
    for g in (W.d1(0), W.d2(n=3000), W.d3(scale=10)):
        s = ht.h_support_graph(g, h, tune=tune)
        assert np.array_equal(s, oracle.h_support(g, h)), (g.name, h, tune)


@pytest.mark.parametrize("make", [
    lambda: gen.complete(9), lambda: gen.cycle(11), lambda: gen.cycle(5), lambda: gen.path(6),
    lambda: gen.star(7), lambda: disjoint_union([gen.complete(5), gen.cycle(9), gen.star(3)])])
@pytest.mark.parametrize("h", [1, 2, 3])
def test_closed_forms_exact(make, h):
    assert_exact(make(), h)


def test_toy_graph_exact():
    import json
    from pathlib import Path
    G = json.loads((Path(__file__).parent / "golden" / "toy14.json").read_text())
    g = from_edge_list(G["n"], G["edges"])
    for h in (1, 2, 3):
        assert_exact(g, h)


@pytest.mark.parametrize("make,h", [
    (lambda: W.d2(n=2000), 1), (lambda: W.d2(n=2000), 2), (lambda: W.d2(n=1000), 3),
    (lambda: W.d3(scale=9), 1), (lambda: W.d3(scale=9), 2), (lambda: W.d3(scale=8), 3),
    (lambda: W.d4_graph((1000, 3, 2, 11)), 2), (lambda: W.d5_graph((500, 2.2, 12.0, 4, 3)), 4)])
def test_scaled_workloads_exact(make, h):
    assert_exact(make(), h)


def test_event_overflow_fallback_exact():
    # a tiny event list forces the full-scan fallback in most rounds
    g = W.d1(2)
    for h in (2, 3):
        t, rho = run_gpu(g, h, tune={"event_capacity": 8, "item_capacity": 8})
        to, ro, _ = oracle.decompose(g, h)
        assert np.array_equal(t, to) and np.array_equal(rho, ro)


def test_edge_cases():
    import paper_2411_06405_amd as ht
    # no edges at all
    g = gen.empty(4)
    t, rho = run_gpu(g, 2)
    assert t.size == 0
    # single edge among isolated vertices; vertex 0 isolated
    g = from_edge_list(7, [[3, 6]])
    for h in (1, 2, 5):
        assert_exact(g, h)
    # h far above the diameter
    assert_exact(gen.cycle(7), 50)


def test_bad_csr_rejected():
    import paper_2411_06405_amd as ht
    g = gen.path(4)
    ci = g.col_idx.copy()
    ci[0], ci[1] = ci[1], ci[0]  # not a valid CSR any more
    with pytest.raises(ht.HotrussError) as ex:
        ht.decompose(g.row_ptr, ci, g.n, 2)
    assert ex.value.status == -2


def test_deterministic():
    g = W.d2(n=2000)
    a = run_gpu(g, 2)
    b = run_gpu(g, 2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("h", [2, 3])
def test_overflow_fallback_small_graph_exact(h):
    # capacities of a few entries force the serial fallback in nearly every round
    g = W.d2(n=1500)
    for cap in (4, 256):
        t, rho = run_gpu(g, h, tune={"event_capacity": cap, "item_capacity": cap})
        to, ro, _ = oracle.decompose(g, h)
        assert np.array_equal(t, to) and np.array_equal(rho, ro), cap


@pytest.mark.parametrize("make", [lambda: W.d2(n=20000), lambda: W.d3(scale=11)])
def test_overflow_fallback_at_scale(make):
    # rows of hundreds of bitset words: the fallback must agree with the
    # work-list path in every round, whichever of the two a round takes
    import paper_2411_06405_amd as ht
    g = make()
    ref_t, ref_r = run_gpu(g, 2, tune={"event_capacity": 1 << 26, "item_capacity": 1 << 26})
    assert ht.last_stats()["overflows"] == 0
    for cap in (4096, 65536):
        t, rho = run_gpu(g, 2, tune={"event_capacity": cap, "item_capacity": cap})
        assert ht.last_stats()["overflows"] > 0
        assert np.array_equal(t, ref_t) and np.array_equal(rho, ref_r), cap


@pytest.mark.parametrize("h", [2, 3])
def test_forced_serial_paths_exact(h):
    # each serial step alone, both together, and overflowing lists
    import paper_2411_06405_amd as ht
    L, S = ht._lib.HO_FLAG_SERIAL_LEVELS, ht._lib.HO_FLAG_SERIAL_SUPPORT
    g = W.d2(n=1500) if h == 2 else W.d2(n=1000)
    to, ro, _ = oracle.decompose(g, h)
    for tune in ({"flags": L}, {"flags": S}, {"flags": L | S}, {"item_capacity": 4},
                 {"event_capacity": 4}, {"item_capacity": 64, "event_capacity": 64}):
        t, rho = run_gpu(g, h, tune=tune)
        assert np.array_equal(t, to) and np.array_equal(rho, ro), tune


def test_host_loop_equals_graph():
    import paper_2411_06405_amd as ht
    g = W.d2(n=5000)
    a = run_gpu(g, 2)
    b = run_gpu(g, 2, tune={"flags": ht._lib.HO_FLAG_HOST_LOOP})
    c = run_gpu(g, 2, tune={"flags": ht._lib.HO_FLAG_STATS})
    st = ht.last_stats()
    assert st["kernel_launches"]["support_update"] == st["rounds"]
    assert st["kernel_ms"]["support_update"] > 0
    for x in (b, c):
        assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1])


@pytest.mark.parametrize("h", [1, 2, 3])
def test_row_compaction_every_launch_exact(h):
    # live slots moved to the front of their rows between graph launches (and
    # between host-driven rounds) at every chance: results unchanged
    import paper_2411_06405_amd as ht
    C = ht._lib.HO_FLAG_COMPACT_EACH
    for g in (W.d1(1), W.d2(n=2000) if h < 3 else W.d2(n=1000), W.d3(scale=9)):
        to, ro, _ = oracle.decompose(g, h)
        for flags in (C, C | ht._lib.HO_FLAG_HOST_LOOP):
            t, rho = run_gpu(g, h, tune={"flags": flags})
            assert np.array_equal(t, to) and np.array_equal(rho, ro), (g.name, flags)


@pytest.mark.parametrize("h", [1, 2, 3])
def test_forced_recovery_with_empty_steps_exact(h):
    # every step re-run from the host, including steps with nothing to do
    # (no events at a level, no support updates) in some rounds
    import paper_2411_06405_amd as ht
    L, S = ht._lib.HO_FLAG_SERIAL_LEVELS, ht._lib.HO_FLAG_SERIAL_SUPPORT
    for g in (W.d1(0), gen.cycle(9), gen.complete(6), gen.star(5), gen.path(4)):
        to, ro, _ = oracle.decompose(g, h)
        for flags in (L | S, S, (L | S) | ht._lib.HO_FLAG_HOST_LOOP):
            t, rho = run_gpu(g, h, tune={"flags": flags})
            assert np.array_equal(t, to) and np.array_equal(rho, ro), (g.name, flags)
