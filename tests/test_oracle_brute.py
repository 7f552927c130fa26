"""The oracle against brute force over all edge subsets (Def. 4), which does
not peel at all, on random graphs with at most 12 vertices."""
import numpy as np
import pytest

from graphgen import gen
from tests.conftest import seeded


@pytest.mark.parametrize("seed", range(60))
def test_oracle_equals_brute_force(oracle_mod, seed):
    rng = seeded(1000 + seed)
    n = int(rng.integers(3, 13))
    g = gen.random_small(n, max_edges=12, seed=seed)
    if g.m == 0:
        return
    for h in (1, 2, 3, 4):
        t, _, _ = oracle_mod.decompose(g, h)
        tb = oracle_mod.brute_trussness(g, h)
        assert np.array_equal(t, tb), (seed, h, t, tb)


@pytest.mark.parametrize("seed", range(20))
def test_support_equals_brute_support(oracle_mod, seed):
    rng = seeded(2000 + seed)
    n = int(rng.integers(3, 13))
    g = gen.random_small(n, max_edges=20, seed=seed)
    if g.m == 0:
        return
    live = rng.random(g.m) < 0.7
    for h in (1, 2, 3):
        s = oracle_mod.h_support(g, h, key=live.astype(np.uint32), thr=1)
        sb = oracle_mod.brute_h_support(g, h, live=live)
        assert np.array_equal(s, sb)
