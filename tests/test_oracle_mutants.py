"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that
the pins catch every one: the pins are strong enough to trust the oracle."""
import numpy as np
import pytest

from graphgen import gen, workloads as W
from tests.test_oracle_h1 import nx_trussness

MUTANTS = {
    "bfs_depth_short": ("if (w->dist[x] == h) continue;", "if (w->dist[x] + 1 == h) continue;"),
    "bfs_depth_long": ("if (w->dist[x] == h) continue;", "if (w->dist[x] == h + 1) continue;"),
    "ball_includes_self": [("w->seen[src] = s; w->dist[src] = 0; w->queue[tail++] = src;",
                            "w->seen[src] = s; w->dist[src] = 0; w->queue[tail++] = src;"
                            " if (mode == 0) w->inball[src] = mark;"),
                           ("return bounded_bfs(g, f, v, h, w, 1, mark, u);",
                            "return bounded_bfs(g, f, v, h, w, 1, mark, UINT32_MAX);")],
    "endpoint_counted": ("else if (w->inball[y] == mark && y != skip) ++count;",
                         "else if (w->inball[y] == mark || y == skip) ++count;"),
    "union_not_intersection": ("else if (w->inball[y] == mark && y != skip) ++count;",
                               "else if (y != skip) ++count;"),
    # removes edges with sup <= k-1 instead of sup <= k-2 (both scans)
    "threshold_off_by_one": [("if ((uint64_t)sup[e] + 2 <= k) R[nr++] = (uint32_t)e;",
                              "if ((uint64_t)sup[e] + 1 <= k) R[nr++] = (uint32_t)e;"),
                             ("if (key[e] && (uint64_t)sup[e] + 2 <= k) R[nr++] = (uint32_t)e;",
                              "if (key[e] && (uint64_t)sup[e] + 1 <= k) R[nr++] = (uint32_t)e;")],
    "level_jump_off_by_one": ("k = mn + 2;", "k = mn + 3;"),
    "trussness_off_by_one": ("t_out[e] = k;", "t_out[e] = k + 1;"),
    "lower_slot_wrong_edge": ("g->slot_eid[j] = g->slot_eid[lo];",
                              "g->slot_eid[j] = g->slot_eid[lo > rp[y] ? lo - 1 : lo];"),
    "ignores_subgraph": ("if (!in_S(f, g->slot_eid[j])) continue;", "(void)0;"),
}


def pins_hold(oracle_mod, lib):
    """Run a battery of pins against a compiled oracle; False on first failure."""
    try:
        for n, h in ((5, 1), (6, 2), (4, 3)):
            if not np.all(oracle_mod.decompose(gen.complete(n), h, lib=lib)[0] == n):
                return False
        for n, h in ((10, 2), (11, 3), (7, 3)):
            exp = 2 * h if n >= 2 * h + 2 else n
            if not np.all(oracle_mod.decompose(gen.cycle(n), h, lib=lib)[0] == exp):
                return False
        for L, h in ((5, 2), (3, 3), (6, 1)):
            if not np.all(oracle_mod.decompose(gen.path(L), h, lib=lib)[0] == min(h, L) + 1):
                return False
        if not np.all(oracle_mod.decompose(gen.star(5), 2, lib=lib)[0] == 6):
            return False
        for seed in range(8):
            g = gen.random_small(9, 11, seed=seed)
            if g.m == 0:
                continue
            for h in (1, 2, 3):
                if not np.array_equal(oracle_mod.decompose(g, h, lib=lib)[0],
                                      oracle_mod.brute_trussness(g, h)):
                    return False
        g = W.d1(0)
        if not np.array_equal(oracle_mod.decompose(g, 1, lib=lib)[0], nx_trussness(g)):
            return False
    except Exception:
        return False
    return True


def test_unmutated_passes(oracle_mod, tmp_path):
    src = oracle_mod.oracle.source_text()
    lib = oracle_mod.oracle.compile_variant(src, tmp_path / "same.so")
    assert pins_hold(oracle_mod, lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(oracle_mod, tmp_path, name):
    edits = MUTANTS[name]
    edits = [edits] if isinstance(edits, tuple) else edits
    src = oracle_mod.oracle.source_text()
    for old, new in edits:
        assert src.count(old) >= 1, name
        src = src.replace(old, new, 1)
    lib = oracle_mod.oracle.compile_variant(src, tmp_path / f"{name}.so")
    assert not pins_hold(oracle_mod, lib), name
