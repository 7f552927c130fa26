"""Pins of the oracle's method-level work count (E_eval, B_alg): a hand-worked
two-round case, a second implementation with networkx breadth-first search,
and the ball-changed rule squeezed between the edges whose h-support really
changes and the safe superset of edges near a removed edge."""
import networkx as nx
import numpy as np
import pytest

import oracle
from graphgen import from_edge_list, gen, workloads as W
from oracle.accounting import count


def test_triangle_with_pendant_by_hand():
    # triangle 0-1-2 plus pendant 2-3, h = 1: round 0 removes (2,3) at k = 2,
    # round 1 the triangle at k = 3.  Worked out from the definitions:
    # evaluations 4 + 2 (the two triangle edges at vertex 2); bytes: 4 initial
    # evaluations of 1+1+4, builds 16+16+20+12, round 0 evaluations 2 x 6 and
    # builds of V_cand = {2, 3} in the triangle, 16 + 8
    g = from_edge_list(4, [[0, 1], [0, 2], [1, 2], [2, 3]])
    t, rho, _ = oracle.decompose(g, 1)
    c = count(g, 1, rho)
    assert c["evaluations"] == 6
    assert c["alg_bytes"] == 24 + 64 + 12 + 24
    assert list(c["a_sizes"]) == [2, 0]


def test_single_round_graphs_evaluate_each_edge_once():
    for g, h in ((gen.complete(6), 2), (gen.cycle(9), 2), (gen.path(5), 1), (gen.star(6), 2)):
        _, rho, info = oracle.decompose(g, h)
        assert info["rounds"] == 1
        assert count(g, h, rho)["evaluations"] == g.m


def _count_networkx(g, h, rho):
    """The same count written with networkx BFS balls, vertex by vertex."""
    n = g.n
    rp, ci = g.row_ptr.astype(int), g.col_idx.astype(int)
    E = [(x, int(ci[j])) for x in range(n) for j in range(rp[x], rp[x + 1]) if ci[j] > x]
    nb = (n + 7) // 8

    def graph(keep):
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(e for e, k in zip(E, keep) if k)
        return G

    def balls(G, j):
        return [set(nx.single_source_shortest_path_length(G, x, cutoff=j)) for x in range(n)]

    def build(G, x):
        ball = nx.single_source_shortest_path_length(G, x, cutoff=h - 1)
        fr = sum(8 + 4 * G.degree(y) for y in ball)
        return min(fr, h * (4 * (n + 1) + 8 * G.number_of_edges() + nb))

    def s(ball):
        return min(4 * (len(ball) - 1), nb)

    G0 = graph([True] * len(E))
    B = balls(G0, h)
    evals = len(E)
    total = sum(s(B[u]) + s(B[v]) + 4 for u, v in E)
    total += sum(build(G0, x) for x in range(n) if G0.degree(x) > 0)
    R = int(rho.max()) + 1
    for r in range(R):
        Gr = graph(rho >= r)
        Gn = graph(rho >= r + 1)
        if Gn.number_of_edges() == 0:
            break
        Bn = balls(Gn, h)
        ch = [B[x] != Bn[x] for x in range(n)]
        for (u, v), k in zip(E, rho >= r + 1):
            if k and (ch[u] or ch[v]):
                evals += 1
                total += s(Bn[u]) + s(Bn[v]) + 4
        ends = {z for (u, v), rr in zip(E, rho) if rr == r for z in (u, v)}
        vc = set()
        for z in ends:
            vc |= set(nx.single_source_shortest_path_length(Gr, z, cutoff=h - 1))
        total += sum(build(Gn, x) for x in vc)
        B = Bn
    return evals, total


@pytest.mark.parametrize("h", [1, 2, 3])
def test_matches_networkx_count(h):
    rng = np.random.default_rng(5)
    for i in range(4):
        n = int(rng.integers(8, 16))
        g = gen.erdos_renyi(n, 0.35, seed=int(rng.integers(1 << 30)))
        if g.m == 0:
            continue
        _, rho, _ = oracle.decompose(g, h)
        c = count(g, h, rho)
        assert (c["evaluations"], c["alg_bytes"]) == _count_networkx(g, h, rho), (i, h)


@pytest.mark.parametrize("h", [2, 3])
def test_ball_changed_rule_between_true_changes_and_safe_superset(h):
    # every edge whose h-support changes between S_r and S_{r+1} is in A_r,
    # and A_r holds only edges with an endpoint within h-1 hops (in S_r) of an
    # endpoint of a removed edge
    g = W.d1(1)
    _, rho, _ = oracle.decompose(g, h)
    c = count(g, h, rho, keep_sets=True)
    rp, ci = g.row_ptr.astype(int), g.col_idx.astype(int)
    E = np.array([(x, int(ci[j])) for x in range(g.n) for j in range(rp[x], rp[x + 1])
                  if ci[j] > x])
    for r, A in enumerate(c["a_sets"]):
        sr = oracle.h_support(g, h, key=rho, thr=r)
        sn = oracle.h_support(g, h, key=rho, thr=r + 1)
        live = rho >= r + 1
        moved = set(np.nonzero(live & (sr != sn))[0])
        assert moved <= set(A), r
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from(tuple(e) for e in E[rho >= r])
        near = set()
        for z in set(E[rho == r].ravel()):
            near |= set(nx.single_source_shortest_path_length(G, int(z), cutoff=h - 1))
        assert all(E[e][0] in near or E[e][1] in near for e in A), r
