"""Input generators: seeded, deterministic, valid simple CSR, canonical edge order."""
import numpy as np
import pytest

from graphgen import concat, disjoint_union, from_edges, gen, validate, workloads as W


@pytest.mark.parametrize("make", [
    lambda: W.d1(0), lambda: W.d2(n=3000), lambda: W.d3(scale=10),
    lambda: W.d4_graph((2000, 4, 2, 9)), lambda: W.d5_graph((500, 2.3, 8.0, 3, 4)),
    lambda: gen.complete(7), lambda: gen.cycle(9), lambda: gen.path(4), lambda: gen.star(5),
    lambda: gen.empty(3)])
def test_valid_and_deterministic(make):
    g1, g2 = make(), make()
    validate(g1)
    assert np.array_equal(g1.row_ptr, g2.row_ptr) and np.array_equal(g1.col_idx, g2.col_idx)
    assert g1.row_ptr.dtype == np.uint32 and g1.col_idx.dtype == np.uint32


def test_canonical_edge_order():
    g = W.d1(3)
    e = g.edges().astype(np.int64)
    assert np.all(e[:, 0] < e[:, 1])
    key = e[:, 0] * g.n + e[:, 1]
    assert np.all(np.diff(key) > 0)
    assert e.shape[0] == g.m


def test_dedup_and_loops_dropped():
    g = from_edges(4, [0, 1, 1, 2, 3, 3], [1, 0, 1, 3, 2, 2])
    assert g.m == 2 and g.edges().tolist() == [[0, 1], [2, 3]]


def test_validate_rejects_asymmetric():
    g = gen.path(3)
    bad = type(g)(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[0] = 2
    with pytest.raises(ValueError):
        validate(bad)


def test_shapes_of_named_workloads():
    g = W.d1(0)
    assert g.n == 200 and 800 < g.m < 1200
    g = W.d3(scale=12)
    assert g.n == 4096
    specs = W.d4_specs()
    assert len(specs) == 512
    assert all(1000 <= n <= 50000 and 3 <= m <= 8 and h in (2, 3) for n, m, h, _ in specs)


def test_union_and_concat_offsets():
    a, b = gen.cycle(5), gen.complete(4)
    u = disjoint_union([a, b])
    assert u.n == 9 and u.m == a.m + b.m
    assert np.array_equal(u.edges()[: a.m], a.edges())
    bt = concat([a, b], [2, 3])
    assert bt.vtx_off.tolist() == [0, 5, 9]
    assert bt.adj_off.tolist() == [0, 10, 22]
    assert bt.edge_off.tolist() == [0, 5, 11]
    assert bt.row_ptr_cat.size == 5 + 1 + 4 + 1
