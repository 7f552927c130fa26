"""At h = 1 the (k,h)-truss is the classical k-truss (Section 2, Def. 1;
Section 3).  networkx's k_truss is an independent implementation."""
import networkx as nx
import numpy as np
import pytest

from graphgen import gen, workloads as W


def nx_trussness(g):
    G = nx.Graph(g.edges().tolist())
    t = {tuple(sorted(e)): 2 for e in G.edges}
    k = 3
    while True:
        T = nx.k_truss(G, k)
        if T.number_of_edges() == 0:
            break
        for e in T.edges:
            t[tuple(sorted(e))] = k
        k += 1
    return np.array([t[(int(u), int(v))] for u, v in g.edges()], dtype=np.uint32)


@pytest.mark.parametrize("make", [lambda: W.d1(0), lambda: W.d1(3), lambda: W.d2(n=1500),
                                  lambda: W.d3(scale=9), lambda: W.d4_graph((1200, 5, 2, 3)),
                                  lambda: gen.complete(8)])
def test_h1_matches_networkx(oracle_mod, make):
    g = make()
    t, _, _ = oracle_mod.decompose(g, 1)
    assert np.array_equal(t, nx_trussness(g))
