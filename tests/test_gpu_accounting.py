"""Work counters of the GPU decomposition against the oracle:
* the method-level count (support evaluations and bytes of the re-evaluating
  peeling method on the same round schedule) that stats mode reports, against
  the oracle's count written from the definitions (dense reachability);
* ball-change events per level (pin P14: every member of every ball leaves
  exactly once; the kernels skip the ball updates of the round that removes
  everything, so the events at level j >= 2 are sum_x |N_G(x,j)| minus the
  same sum over the edges of that last round), against oracle BFS balls."""
import numpy as np
import pytest

import oracle
from graphgen import gen, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [(lambda: W.d1(0), 1), (lambda: W.d1(0), 2), (lambda: W.d1(1), 3),
         (lambda: W.d3(scale=9), 2), (lambda: W.d2(n=1000), 2), (lambda: W.d2(n=800), 3),
         (lambda: gen.cycle(11), 2)]


@pytest.mark.parametrize("make,h", CASES)
def test_method_work_count_matches_oracle(make, h):
    import paper_2411_06405_amd as ht
    g = make()
    print(f"[gpu] work count {g.name} n={g.n} m={g.m} h={h}", flush=True)
    t, rho = ht.decompose_graph(g, h, tune={"flags": ht._lib.HO_FLAG_STATS})
    st = ht.last_stats()
    to, ro, _ = oracle.decompose(g, h)
    assert np.array_equal(t, to) and np.array_equal(rho, ro)
    c = oracle.accounting.count(g, h, ro)
    assert st["evaluations"] == c["evaluations"]
    assert st["alg_bytes"] == c["alg_bytes"]


def _ball_total(g, h, keep):
    """sum_x |N_S(x,h)| over the kept edges, by dense reachability."""
    from oracle.accounting import _edges, _reach
    eu, ev = _edges(g)
    R = _reach(g.n, eu, ev, keep, h)
    return int(R.sum()) - g.n


@pytest.mark.parametrize("make,h", CASES + [(lambda: W.d3(scale=10), 3)])
def test_events_per_level_p14(make, h):
    import paper_2411_06405_amd as ht
    g = make()
    print(f"[gpu] events per level {g.name} n={g.n} m={g.m} h={h}", flush=True)
    t, rho = ht.decompose_graph(g, h)
    ev = ht.last_stats()["level_events"]
    last = rho == rho.max()
    every = np.ones(g.m, dtype=bool)
    assert ev[0] == 2 * g.m
    for j in range(2, h + 1):
        assert ev[j - 1] == _ball_total(g, j, every) - _ball_total(g, j, last), j
