"""Pins of the H-index fixpoint oracle (Section 4.1: the H-index operator, the
h-hop reachable path key, the higher-order H-index sequence, Theorems 1-2).
None of the expected values below comes from the function under test."""
import itertools

import networkx as nx
import numpy as np
import pytest

from graphgen import disjoint_union, from_edges, gen, workloads as W
from oracle import brute_trussness, decompose, h_support
from oracle.hindex import UNREACHED, hindex, hindex_sequence, hindex_trussness, path_keys
from tests.conftest import seeded


@pytest.mark.parametrize("vals,y", [
    ([], 0), ([0, 0, 0], 0), ([100], 1), ([3, 0, 6, 1, 5], 3), ([1, 3, 1], 1),
    ([4, 4, 4, 4], 4), ([25, 8, 5, 3, 3], 3), ([10, 8, 5, 4, 3], 4), ([2, 2], 2),
    ([1, 1, 1, 1], 1), ([5, 5, 5, 5, 5, 5], 5), ([0, 7], 1),
])
def test_hindex_operator(vals, y):
    # textbook H-index values, worked by hand
    assert hindex(vals) == y


@pytest.mark.parametrize("seed", range(10))
def test_path_keys_against_simple_paths(seed):
    # Def. of P: max over simple paths of <= h edges of the min key, by
    # enumerating every simple path with networkx
    rng = seeded(100 + seed)
    n = int(rng.integers(4, 8))
    g = gen.erdos_renyi(n, float(rng.uniform(0.3, 0.7)), seed=seed)
    ends = g.edges().astype(np.int64)
    key = rng.integers(0, 6, size=g.m)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    kmap = {}
    for i, (a, b) in enumerate(ends.tolist()):
        G.add_edge(a, b)
        kmap[(a, b)] = kmap[(b, a)] = int(key[i])
    for h in (1, 2, 3):
        for x in range(n):
            p = path_keys(n, ends, key, h, x)
            for w in range(n):
                if w == x:
                    continue
                best = UNREACHED
                for path in nx.all_simple_paths(G, x, w, cutoff=h):
                    best = max(best, min(kmap[(a, b)] for a, b in zip(path, path[1:])))
                assert p[w] == best, (seed, h, x, w)


def test_hand_worked_sequences():
    # diamond (K4 minus an edge), h = 1: the middle edge has two triangles but
    # lies in no 4-truss; one sweep lowers it, the next changes nothing
    g = from_edges(4, [0, 0, 1, 1, 2], [1, 2, 2, 3, 3])
    seq = hindex_sequence(g, 1)
    assert [s.tolist() for s in seq] == [[1, 1, 2, 1, 1], [1, 1, 1, 1, 1], [1, 1, 1, 1, 1]]
    # path 0-1-2-3-4, h = 2: sup_G = 1, 2, 2, 1; the inner edges see one common
    # neighbour on each side but only one of them through keys >= 2
    seq = hindex_sequence(gen.path(4), 2)
    assert [s.tolist() for s in seq] == [[1, 2, 2, 1], [1, 1, 1, 1], [1, 1, 1, 1]]


@pytest.mark.parametrize("h", [1, 2, 3])
def test_closed_forms_converge_at_once(h):
    # complete graphs, long cycles and stars start at their fixpoint: sup = t-2
    for g, t in ((gen.complete(6), 6), (gen.cycle(2 * h + 4), 2 * h if h > 1 else 2)):
        seq = hindex_sequence(g, h)
        assert len(seq) == 2 and np.all(seq[-1] == t - 2)
    if h >= 2:
        seq = hindex_sequence(gen.star(5), h)
        assert len(seq) == 2 and np.all(seq[-1] == 4)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("h", [1, 2, 3])
def test_converges_to_trussness(seed, h):
    # Theorem 2 against the peeling oracle; Theorem 1 (non-increasing) and the
    # lower bound t-2 along the way; H^(0) is the h-support
    g = W.d1(seed)
    t, _, _ = decompose(g, h)
    seq = hindex_sequence(g, h)
    assert np.array_equal(seq[0], h_support(g, h).astype(np.int64))
    for a, b in zip(seq, seq[1:]):
        assert np.all(b <= a)
        assert np.all(b >= t.astype(np.int64) - 2)
    assert np.array_equal(seq[-1] + 2, t.astype(np.int64))
    assert np.array_equal(seq[-1], seq[-2])
    assert not any(np.array_equal(a, b) for a, b in zip(seq[:-2], seq[1:-1]))


@pytest.mark.parametrize("seed", range(6))
def test_tiny_graphs_against_brute_force(seed):
    rng = seeded(200 + seed)
    n = int(rng.integers(5, 9))
    g = gen.erdos_renyi(n, float(rng.uniform(0.3, 0.6)), seed=seed)
    for h in (1, 2, 3):
        t, _ = hindex_trussness(g, h)
        assert np.array_equal(t.astype(np.int64), brute_trussness(g, h).astype(np.int64))


def test_h1_is_the_triangle_edge_pair_iteration():
    # h = 1 reduces to the k-truss H-index of the prior work (Section 4.1):
    # H^(n)(e) = H({min(H(e1), H(e2)) : (e1, e2) a triangle edge pair of e})
    g = W.d1(3)
    ends = [tuple(e) for e in g.edges().tolist()]
    idx = {e: i for i, e in enumerate(ends)}
    G = nx.Graph(ends)
    pairs = []
    for u, v in ends:
        pairs.append([(idx[tuple(sorted((u, w)))], idx[tuple(sorted((v, w)))])
                      for w in nx.common_neighbors(G, u, v)])
    H = np.array([len(p) for p in pairs], dtype=np.int64)
    seq = hindex_sequence(g, 1)
    for step in seq[1:]:
        H = np.array([hindex([min(H[a], H[b]) for a, b in p]) for p in pairs], dtype=np.int64)
        assert np.array_equal(step, H)


def test_empty_isolated_and_union():
    assert len(hindex_sequence(gen.empty(4), 2)) == 1
    g = from_edges(5, [0], [4])
    t, sweeps = hindex_trussness(g, 2)
    assert t.tolist() == [2] and sweeps == 1
    parts = [gen.complete(5), gen.path(3), gen.cycle(7)]
    u = disjoint_union(parts)
    tu, _ = hindex_trussness(u, 2)
    assert np.array_equal(tu, np.concatenate([hindex_trussness(p, 2)[0] for p in parts]))


def test_max_sweeps_truncates():
    g = W.d1(0)
    full = hindex_sequence(g, 2)
    assert len(full) > 3
    part = hindex_sequence(g, 2, max_sweeps=2)
    assert len(part) == 3
    for a, b in zip(part, full):
        assert np.array_equal(a, b)
