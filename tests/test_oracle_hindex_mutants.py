"""Plant plausible mistakes in a copy of the H-index oracle (on the CPU) and
check that its pins catch every one: the pins are strong enough to trust the
H-index oracle the GPU sweeps are compared with."""
import importlib.util
import sys
from pathlib import Path

import networkx as nx
import numpy as np
import pytest

from graphgen import from_edges, gen, workloads as W
from oracle import decompose

SRC = Path(__file__).resolve().parents[1] / "oracle" / "hindex.py"

MUTANTS = {
    # one hop too many or too few in the path keys
    "hops_plus_one": ("    for _ in range(h):\n        q = p.copy()",
                      "    for _ in range(h + 1):\n        q = p.copy()"),
    "hops_minus_one": ("    for _ in range(h):\n        q = p.copy()",
                       "    for _ in range(max(h - 1, 1)):\n        q = p.copy()"),
    # the path key takes the largest edge on the path instead of the smallest
    "key_max_not_min": ("np.maximum.at(q, b[ok], np.minimum(p[a[ok]], k[ok]))",
                        "np.maximum.at(q, b[ok], np.maximum(p[a[ok]], k[ok]))"),
    # the hop bound is ignored (widest paths of any length)
    "hop_bound_ignored": ("    for _ in range(h):\n        q = p.copy()",
                          "    for _ in range(n):\n        q = p.copy()"),
    # the endpoints are counted among the common neighbours (a vertex keeps a
    # key to itself and the exclusion is dropped)
    "endpoints_counted": [("        common[u] = common[v] = False\n", ""),
                          ("    p[src] = UNREACHED\n    return p", "    return p")],
    # H-index operator off by one
    "hindex_off_by_one": ("while y < s.size and s[y] >= y + 1:", "while y < s.size and s[y] >= y:"),
    # min of the two keys replaced by max
    "pair_max_not_min": ("out[i] = hindex(np.minimum(pu[common], pv[common]))",
                         "out[i] = hindex(np.maximum(pu[common], pv[common]))"),
    # the sequence starts from the triangle count instead of the h-support
    "start_from_h1": ("    H = h_support(g, h).astype(np.int64)", "    H = h_support(g, 1).astype(np.int64)"),
    # stops one sweep early (the sweep that changes nothing is not run)
    "stops_early": ("        if np.array_equal(nxt, seq[-2]) or (max_sweeps and len(seq) - 1 >= max_sweeps):",
                    "        if len(seq) >= 3 or (max_sweeps and len(seq) - 1 >= max_sweeps):"),
}


def load_mutant(name, edits, tmp_path):
    text = SRC.read_text()
    for old, new in ([edits] if isinstance(edits[0], str) else edits):
        assert text.count(old) == 1, (name, old)
        text = text.replace(old, new)
    # the copy imports h_support from the real oracle package
    text = text.replace("from .oracle import h_support", "from oracle import h_support")
    path = tmp_path / f"hindex_{name}.py"
    path.write_text(text)
    spec = importlib.util.spec_from_file_location(f"hindex_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


def pins_hold(mod) -> bool:
    """The pins of test_oracle_hindex, condensed; False on the first failure."""
    try:
        if [mod.hindex(v) for v in ([3, 0, 6, 1, 5], [1, 3, 1], [4, 4, 4, 4], [0, 7])] != [3, 1, 4, 1]:
            return False
        diamond = from_edges(4, [0, 0, 1, 1, 2], [1, 2, 2, 3, 3])
        if [s.tolist() for s in mod.hindex_sequence(diamond, 1)] != \
                [[1, 1, 2, 1, 1], [1, 1, 1, 1, 1], [1, 1, 1, 1, 1]]:
            return False
        if [s.tolist() for s in mod.hindex_sequence(gen.path(4), 2)] != \
                [[1, 2, 2, 1], [1, 1, 1, 1], [1, 1, 1, 1]]:
            return False
        # path keys against every simple path on a small graph
        rng = np.random.default_rng(7)
        g = gen.erdos_renyi(7, 0.5, seed=3)
        ends = g.edges().astype(np.int64)
        key = rng.integers(0, 6, size=g.m)
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        kmap = {}
        for i, (a, b) in enumerate(ends.tolist()):
            G.add_edge(a, b)
            kmap[(a, b)] = kmap[(b, a)] = int(key[i])
        for h in (1, 2, 3):
            for x in range(g.n):
                p = mod.path_keys(g.n, ends, key, h, x)
                for w in range(g.n):
                    if w == x:
                        continue
                    best = -1
                    for path in nx.all_simple_paths(G, x, w, cutoff=h):
                        best = max(best, min(kmap[(a, b)] for a, b in zip(path, path[1:])))
                    if p[w] != best:
                        return False
        # Theorem 2 and the lower bound on a random graph
        g = W.d1(0)
        for h in (1, 2):
            t = decompose(g, h)[0].astype(np.int64)
            seq = mod.hindex_sequence(g, h)
            if not np.array_equal(seq[-1] + 2, t) or not np.array_equal(seq[-1], seq[-2]):
                return False
            if any(np.any(s < t - 2) for s in seq):
                return False
    except (AssertionError, IndexError, ValueError):
        return False
    return True


def test_real_oracle_passes_the_battery():
    import oracle.hindex as real
    assert pins_hold(real)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    mod = load_mutant(name, MUTANTS[name], tmp_path)
    assert not pins_hold(mod), f"planted mistake {name} passed every pin"
