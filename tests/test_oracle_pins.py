"""The oracle against closed forms and invariants fixed by the definitions
(Section 2, Defs. 3-4; Section 3, Lemma 1).  None of these expected values is
produced by the oracle itself."""
import networkx as nx
import numpy as np
import pytest

from graphgen import disjoint_union, from_edges, gen, workloads as W
from tests.conftest import seeded


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 9])
@pytest.mark.parametrize("h", [1, 2, 3, 5])
def test_complete_graph(oracle_mod, n, h):
    # K_n: every ball is the rest of the graph, sup = n-2, so t = n
    t, rho, info = oracle_mod.decompose(gen.complete(n), h)
    assert np.all(t == n)
    assert info["rounds"] == 1


@pytest.mark.parametrize("n", range(3, 13))
@pytest.mark.parametrize("h", [1, 2, 3])
def test_cycle(oracle_mod, n, h):
    # C_n: ball = h vertices each side; for n >= 2h+2 the common part of two
    # adjacent balls has 2h-2 vertices, so t = 2h; smaller cycles saturate.
    t, _, _ = oracle_mod.decompose(gen.cycle(n), h)
    expect = 2 * h if n >= 2 * h + 2 else n
    if h == 1:
        expect = 3 if n == 3 else 2
    assert np.all(t == expect), (n, h, t)


@pytest.mark.parametrize("L", range(1, 9))
@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_path(oracle_mod, L, h):
    t, _, _ = oracle_mod.decompose(gen.path(L), h)
    assert np.all(t == min(h, L) + 1), (L, h, t)


@pytest.mark.parametrize("r", [1, 2, 3, 6, 10])
def test_star(oracle_mod, r):
    # h=1: no triangles, t=2; h>=2: leaves are common 2-hop neighbours through
    # the centre, sup = r-1, t = r+1
    t1, _, _ = oracle_mod.decompose(gen.star(r), 1)
    assert np.all(t1 == 2)
    for h in (2, 3):
        t, _, _ = oracle_mod.decompose(gen.star(r), h)
        assert np.all(t == r + 1)


@pytest.mark.parametrize("seed", range(12))
def test_diameter_saturation(oracle_mod, seed):
    # connected G with diameter <= h: every ball is V minus the vertex, so t = n
    rng = seeded(seed)
    n = int(rng.integers(4, 30))
    g = gen.erdos_renyi(n, float(rng.uniform(0.2, 0.6)), seed=seed)
    G = nx.Graph(g.edges().tolist())
    G.add_nodes_from(range(n))
    if not nx.is_connected(G):
        pytest.skip("disconnected draw")
    d = nx.diameter(G)
    for h in (d, d + 1):
        t, _, _ = oracle_mod.decompose(g, h)
        assert np.all(t == n)


def test_empty_and_isolated(oracle_mod):
    t, rho, info = oracle_mod.decompose(gen.empty(5), 2)
    assert t.size == 0 and info["rounds"] == 0
    g = from_edges(6, [0], [5])   # single edge plus isolated vertices
    for h in (1, 2, 7):
        t, _, _ = oracle_mod.decompose(g, h)
        assert t.tolist() == [2]


def test_disjoint_union(oracle_mod):
    # distance across components is infinite: components decompose independently
    parts = [W.d1(1), gen.complete(6), gen.cycle(11), gen.star(4), gen.path(3)]
    u = disjoint_union(parts)
    for h in (1, 2, 3):
        tu, _, _ = oracle_mod.decompose(u, h)
        tp = np.concatenate([oracle_mod.decompose(p, h)[0] for p in parts])
        assert np.array_equal(tu, tp)


@pytest.mark.parametrize("seed", range(3))
def test_bounds_and_monotonicity(oracle_mod, seed):
    # 2 <= t(e,h) <= sup_G(e,h)+2, t(e,h) <= t(e,h+1), t <= |component|
    g = W.d1(seed)
    G = nx.Graph(g.edges().tolist())
    comp = {v: len(c) for c in nx.connected_components(G) for v in c}
    prev = None
    for h in (1, 2, 3, 4):
        t, rho, info = oracle_mod.decompose(g, h)
        sup = oracle_mod.h_support(g, h)
        assert np.all(t >= 2) and np.all(t <= sup.astype(np.int64) + 2)
        cs = np.array([comp[int(u)] for u, _ in g.edges()])
        assert np.all(t <= cs)
        if prev is not None:
            assert np.all(t >= prev)
        prev = t
        # rounds: k never decreases, rounds are dense
        rk = info["round_k"]
        assert np.all(np.diff(rk.astype(np.int64)) >= 0)
        assert set(np.unique(rho).tolist()) == set(range(info["rounds"]))


def test_h_support_h1_is_triangle_count(oracle_mod):
    # Section 2: sup_G(e) = |N(u) ∩ N(v)|, the number of triangles on e
    g = W.d1(2)
    G = nx.Graph(g.edges().tolist())
    sup = oracle_mod.h_support(g, 1)
    for i, (u, v) in enumerate(g.edges().tolist()):
        assert sup[i] == len(set(G[u]) & set(G[v]))


def test_h_support_against_networkx_distances(oracle_mod):
    # Def. 3 from networkx shortest paths (an independent BFS)
    g = W.d1(4)
    G = nx.Graph(g.edges().tolist())
    for h in (2, 3):
        sup = oracle_mod.h_support(g, h)
        ball = {x: {y for y, d in nx.single_source_shortest_path_length(G, x, cutoff=h).items()
                    if y != x} for x in G.nodes}
        for i, (u, v) in enumerate(g.edges().tolist()):
            assert sup[i] == len(ball[u] & ball[v])


def test_h_support_subgraph_filter(oracle_mod):
    # sup_S uses distances in S only: drop a random half of the edges
    g = W.d1(0)
    rng = seeded(5)
    key = (rng.random(g.m) < 0.5).astype(np.uint32)
    E = g.edges().tolist()
    G = nx.Graph([E[i] for i in range(g.m) if key[i]])
    sup = oracle_mod.h_support(g, 2, key=key, thr=1)
    for i, (u, v) in enumerate(E):
        if not key[i]:
            assert sup[i] == 0
            continue
        bu = set(nx.single_source_shortest_path_length(G, u, cutoff=2)) - {u}
        bv = set(nx.single_source_shortest_path_length(G, v, cutoff=2)) - {v}
        assert sup[i] == len(bu & bv)


def test_sampled_support_matches_full(oracle_mod):
    # entry-point consistency (not a pin): the sampled evaluation used at full
    # benchmark sizes returns the full evaluation's values on its edges
    g = W.d2(n=2000)
    for h in (1, 2, 3):
        full = oracle_mod.h_support(g, h)
        e = np.random.default_rng(h).choice(g.m, 50, replace=False).astype(np.uint32)
        assert np.array_equal(oracle_mod.h_support_edges(g, h, e), full[e])
