"""The truss-extraction oracle against closed forms and a separately written
union-find (the (k,h)-truss is {e : t(e,h) >= k}, Def. 4)."""
import numpy as np
import pytest

from graphgen import disjoint_union, gen, workloads as W

NONE = 0xFFFFFFFF


def _uf_components(g, t, k):
    """Plain Python union-find over the truss edges (independent of scipy)."""
    parent = list(range(g.n))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x
    e = g.edges()
    for (u, v), te in zip(e.tolist(), np.asarray(t).tolist()):
        if te >= k:
            a, b = find(u), find(v)
            if a != b:
                parent[max(a, b)] = min(a, b)
    label = np.full(g.m, NONE, dtype=np.uint32)
    roots = set()
    for i, ((u, v), te) in enumerate(zip(e.tolist(), np.asarray(t).tolist())):
        if te >= k:
            label[i] = find(u)
            roots.add(find(u))
    return label, len(roots)


def test_cliques_closed_form(oracle_mod):
    # K5 + K4: t = 5 on the K5 edges and 4 on the K4 edges for every h (K_n
    # has t = n, components are independent)
    g = disjoint_union([gen.complete(5), gen.complete(4)])
    t = np.array([5 if max(u, v) < 5 else 4 for u, v in g.edges().tolist()], dtype=np.uint32)
    for k, count in ((2, 2), (4, 2), (5, 1), (6, 0)):
        lab, c = oracle_mod.truss_components(g, t, k)
        assert c == count
        assert np.all(lab[t < k] == NONE)
        assert np.all(lab[(t >= k) & (t == 5)] == 0)
        assert np.all(lab[(t >= k) & (t == 4)] == 5)


@pytest.mark.parametrize("L,h", [(5, 1), (5, 2), (3, 4)])
def test_path_closed_form(oracle_mod, L, h):
    # a path with L edges has t = min(h, L) + 1 on every edge: one component
    g = gen.path(L)
    t = np.full(g.m, min(h, L) + 1, dtype=np.uint32)
    lab, c = oracle_mod.truss_components(g, t, min(h, L) + 1)
    assert c == 1 and np.all(lab == 0)
    lab, c = oracle_mod.truss_components(g, t, min(h, L) + 2)
    assert c == 0 and np.all(lab == NONE)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("h", [1, 2])
def test_against_union_find_and_nesting(oracle_mod, seed, h):
    g = disjoint_union([W.d1(seed % 5), gen.cycle(7), gen.complete(6)])
    t, _, _ = oracle_mod.decompose(g, h)
    prev = None
    for k in range(2, int(t.max()) + 2):
        lab, c = oracle_mod.truss_components(g, t, k)
        ref, rc = _uf_components(g, t, k)
        assert c == rc and np.array_equal(lab, ref), k
        if prev is not None:
            # the truss at k lies inside the truss at k-1, component by component
            inside = lab != NONE
            assert np.all(prev[inside] != NONE)
            for comp in np.unique(lab[inside]):
                assert np.unique(prev[lab == comp]).size == 1
        prev = lab
