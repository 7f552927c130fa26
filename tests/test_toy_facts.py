"""The facts printed about the paper's toy network (Section 1, Example 1;
Section 3, Example 2) hold on tests/golden/toy14.json, a graph built to match
them.  These facts separate the readings used here (balls exclude their own
vertex; paths may pass through the endpoints) from the alternatives."""
import json
from pathlib import Path

import numpy as np

from graphgen import from_edge_list

G = json.loads((Path(__file__).parent / "golden" / "toy14.json").read_text())


def test_toy_facts(oracle_mod):
    g = from_edge_list(G["n"], G["edges"])
    f = G["facts"]
    t1, _, _ = oracle_mod.decompose(g, 1)
    assert sorted(set(t1.tolist())) == f["h1_trussness_values"]
    t2, _, _ = oracle_mod.decompose(g, 2)
    assert sorted(set(t2.tolist())) == f["h2_trussness_values"]
    E = [tuple(e) for e in g.edges().tolist()]
    e = E.index(tuple(f["min_initial_2_support_edge"]))
    s = oracle_mod.h_support(g, 2)
    assert s[e] == f["min_initial_2_support"] == s.min()
    assert (s == s.min()).sum() == 1
    assert t2[e] == f["min_edge_2_trussness"]
    key = np.ones(g.m, np.uint32)
    key[e] = 0
    s2 = oracle_mod.h_support(g, 2, key=key, thr=1)
    changed = sorted(E[i] for i in np.nonzero((s2 != s) & (key == 1))[0])
    assert changed == [tuple(x) for x in f["changed_after_removal"]]


def test_toy_reading_endpoints_counted_breaks_f3(oracle_mod):
    # if balls included their own vertex, (v3,v6) would count v3 and v6 too
    g = from_edge_list(G["n"], G["edges"])
    s = oracle_mod.h_support(g, 2)
    E = [tuple(e) for e in g.edges().tolist()]
    e = E.index(tuple(G["facts"]["min_initial_2_support_edge"]))
    assert s[e] + 2 != G["facts"]["min_initial_2_support"]
