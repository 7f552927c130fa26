"""The exactness certificate accepts true decompositions and rejects
perturbed ones (single-edge +-1, whole-round level shifts, swapped rounds)."""
import numpy as np
import pytest

from graphgen import gen, workloads as W
from tests.conftest import seeded


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("h", [1, 2, 3])
def test_accepts_oracle_output(oracle_mod, seed, h):
    g = W.d1(seed)
    t, rho, _ = oracle_mod.decompose(g, h)
    ok, info = oracle_mod.certify(g, h, t, rho)
    assert ok, info
    # sampled form
    ok, info = oracle_mod.certify(g, h, t, rho, sample=np.arange(0, g.m, 7))
    assert ok


@pytest.mark.parametrize("h", [1, 2, 3])
def test_rejects_single_edge_changes(oracle_mod, h):
    g = W.d1(1)
    t, rho, info = oracle_mod.decompose(g, h)
    rng = seeded(h)
    for e in rng.choice(g.m, size=25, replace=False):
        for d in (-1, 1):
            if int(t[e]) + d < 2:
                continue
            t2 = t.copy()
            t2[e] = int(t[e]) + d
            ok, _ = oracle_mod.certify(g, h, t2, rho)
            assert not ok


@pytest.mark.parametrize("h", [2, 3])
def test_rejects_whole_round_shift(oracle_mod, h):
    # shifting every edge of one round keeps C0 consistent when neighbours allow
    g = W.d1(2)
    t, rho, info = oracle_mod.decompose(g, h)
    R = info["rounds"]
    rejected = 0
    for r in range(R):
        for d in (-1, 1):
            t2 = t.astype(np.int64)
            t2[rho == r] += d
            if t2.min() < 2:
                continue
            t2 = t2.astype(np.uint32)
            ok, _ = oracle_mod.certify(g, h, t2, rho)
            rejected += (not ok)
            assert not ok
    assert rejected > 0


def test_rejects_swapped_rounds(oracle_mod):
    g = W.d1(0)
    t, rho, info = oracle_mod.decompose(g, 2)
    rho2 = rho.copy()
    a, b = rho == 0, rho == info["rounds"] - 1
    rho2[a], rho2[b] = info["rounds"] - 1, 0
    ok, _ = oracle_mod.certify(g, 2, t, rho2)
    assert not ok


def test_accepts_other_valid_schedule(oracle_mod):
    # one edge per round in removal order of Algorithm 1 is also a schedule
    g = gen.cycle(9)
    t, rho, _ = oracle_mod.decompose(g, 2)
    ok, _ = oracle_mod.certify(g, 2, t, rho)
    assert ok
